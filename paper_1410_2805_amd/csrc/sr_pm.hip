// Long-range particle-mesh force (Sec. 2.3) on one GPU.
//
//   deposit   CIC weights from FP64 grid coordinates; every particle adds its
//             8 contributions to a 64-bit fixed-point grid with integer
//             atomics (neighbouring lanes share their common corners
//             first), so the density is independent of arrival order.
//   FFT       radix-4 (and one radix-2) Stockham passes in LDS along z, y
//             and x; the twiddles are an FP64-built float32 table.  The
//             first pass reads the fixed-point sums directly.
//   k space   applied inside the x pass, between its forward and inverse
//             transforms: 4 pi G_6 S (Eqs. (greenf), (filter)) and the
//             Super-Lanczos gradient (Eq. (sldiff)) give two spectra, A_x +
//             i A_y and A_z.  Each A_d is the transform of a real field, so
//             one complex inverse FFT returns a_x and a_y together.
//   interp    CIC gather of (a_x, a_y, a_z) at each particle.
//
// Eight launches per force: mass maximum, deposit, z, y, x (forward, k
// space, inverse), y and z (inverse, both grids), interpolation.
//
// All k-space factors are separable per axis except the G_6 sum; per-axis
// tables are built in FP64 on the host.  The G_6 axis term is stored minus
// its k = 0 value, so the small-k denominator carries no cancellation.
#include <climits>
#include <cmath>
#include <vector>

#include "sr_internal.h"
#include "sr_pm.h"
#include "sr_split.h"

struct sr_pm {
    sr_ctx *ctx = nullptr;
    int ng = 0, log2ng = 0;
    double len = 0.0, delta = 0.0;
    float sigma = 0.f;
    int ns = 0;
    float2 *ga = nullptr;   // complex grid; density, then A_x + i A_y
    float2 *gb = nullptr;   // complex grid; A_z
    unsigned long long *acc = nullptr;  // 64-bit fixed-point deposit, zero between calls
    float2 *tw = nullptr;   // [ng] exp(-2 pi i m / ng)
    float *tab = nullptr;   // [3 ng] G_6 axis term, filter factor, gradient factor
    unsigned *part = nullptr;  // per-block maxima of the masses (bit patterns)
};

namespace {

constexpr int kBlock = 256;
constexpr int kFftThreads = 256;
constexpr int kFftElems = 2048;  // complex values per FFT block (lines x ng)
constexpr int kStatusMass = 2;   // status bit: negative / non-finite mass or position

struct PmGeo {
    double scale;  // ng / len: grid coordinate per unit length
    int ng;
    int log2ng;
};

// Position sources: global float32 coordinates, or split coordinates.
struct SrcGlobal {
    const float *x, *y, *z;
    __device__ __forceinline__ void get(int i, double p[3]) const
    {
        p[0] = x[i];
        p[1] = y[i];
        p[2] = z[i];
    }
};

struct SrcSplit {
    const int *cell3;
    const float *ox, *oy, *oz;
    double h[3];
    __device__ __forceinline__ void get(int i, double p[3]) const
    {
        const int c = cell3[i];
        p[0] = (double)(c & 1023) * h[0] + (double)ox[i];
        p[1] = (double)((c >> 10) & 1023) * h[1] + (double)oy[i];
        p[2] = (double)((c >> 20) & 1023) * h[2] + (double)oz[i];
    }
};

// CIC cell and fractions of one particle (periodic).  False for a
// non-finite coordinate.
__device__ __forceinline__ bool cic_setup(const double p[3], const PmGeo &g, int i0[3],
                                          int i1[3], double f[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = p[d] * g.scale;
        if (!isfinite(u))
            return false;
        u -= (double)g.ng * floor(u / (double)g.ng);
        const double fl = floor(u);
        f[d] = u - fl;
        int c = (int)fl;
        c = c >= g.ng ? c - g.ng : (c < 0 ? c + g.ng : c);
        i0[d] = c;
        i1[d] = c + 1 == g.ng ? 0 : c + 1;
    }
    return true;
}

// Fixed-point shift S: every particle's mass is below 2^em, n <= 2^en, so
// the sum of all contributions scaled by 2^S stays below 2^62.
__device__ __forceinline__ int fixed_shift(unsigned mbits, int n)
{
    if (mbits == 0u)
        return 0;
    int em;
    (void)frexpf(__uint_as_float(mbits), &em);
    const int en = n > 1 ? 32 - __clz(n - 1) : 0;
    return 62 - em - en;
}

__device__ __forceinline__ unsigned wave_max(unsigned v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = max(v, (unsigned)__shfl_xor((int)v, off));
    return v;
}

// Largest mass from the per-block partial maxima (wave-uniform result).
__device__ __forceinline__ unsigned parts_max(const unsigned *__restrict__ part, int nparts)
{
    unsigned v = 0u;
    for (int k = threadIdx.x & 63; k < nparts; k += 64)
        v = max(v, part[k]);
    return wave_max(v);
}

// Per-block maxima of the masses (the bit pattern of a non-negative float
// orders like its value); a negative or non-finite mass sets the status.
// No atomics on one word: each block writes its own partial.  Each thread
// keeps kMaxUnroll independent loads in flight.
constexpr int kMaxUnroll = 8;

__global__ __launch_bounds__(kBlock) void k_pm_mass_max(const float *__restrict__ m, int n,
                                                        unsigned *__restrict__ part,
                                                        int *__restrict__ status)
{
    __shared__ unsigned sh[kBlock / 64];
    unsigned v = 0u;
    bool bad = false;
    for (int base = blockIdx.x * kBlock * kMaxUnroll + threadIdx.x; base < n;
         base += gridDim.x * kBlock * kMaxUnroll) {
        float mv[kMaxUnroll];
#pragma unroll
        for (int u = 0; u < kMaxUnroll; ++u) {
            const int i = base + u * kBlock;
            mv[u] = i < n ? m[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < kMaxUnroll; ++u) {
            if (!(mv[u] >= 0.f) || !isfinite(mv[u]))
                bad = true;
            else
                v = max(v, __float_as_uint(mv[u]));
        }
    }
    if (bad)
        atomicOr(status, kStatusMass);
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned b = sh[0];
        for (int w = 1; w < kBlock / 64; ++w)
            b = max(b, sh[w]);
        part[blockIdx.x] = b;
    }
}

__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, int d)
{
    const int lo = __shfl_up((int)(unsigned)v, d), hi = __shfl_up((int)(unsigned)(v >> 32), d);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Deposit: each block takes kDepBlock consecutive particles and their 8
// fixed-point CIC contributions each.  When the block's particles fill a
// small box of grid points (input in lattice or cell order does), the block
// sums into a dense LDS window over that box first (64-bit LDS atomics) and
// then adds each non-zero window point to the grid once.  Otherwise every
// contribution goes to the grid directly, where along z the upper corners of
// lane k are the lower corners of lane k + 1 whenever the two particles sit
// in neighbouring cells of one (x, y) column, so lane k + 1 takes those four
// values over by a lane shuffle and one atomic serves both.  Integer sums
// make the result independent of every order.
constexpr int kDepPer = 2;                    // particles per thread
constexpr int kDepBlock = kBlock * kDepPer;   // particles per block
constexpr int kWin = 6144;                    // LDS window points (48 KiB)

template <class Src>
__global__ __launch_bounds__(kBlock) void k_pm_deposit(Src src, const float *__restrict__ m, int n,
                                                       PmGeo g, const unsigned *__restrict__ part,
                                                       int nparts,
                                                       unsigned long long *__restrict__ acc,
                                                       int *__restrict__ status)
{
    __shared__ unsigned long long win[kWin];
    __shared__ int red[6][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int shift = fixed_shift(parts_max(part, nparts), n);
    bool ok[kDepPer];
    double f[kDepPer][3], q[kDepPer];
    int i0[kDepPer][3], i1[kDepPer][3];
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {-1, -1, -1};
#pragma unroll
    for (int k = 0; k < kDepPer; ++k) {
        const int i = blockIdx.x * kDepBlock + k * kBlock + threadIdx.x;
        ok[k] = false;
        q[k] = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            f[k][d] = 0.0;
            i0[k][d] = i1[k][d] = 0;
        }
        if (i < n) {
            double p[3];
            src.get(i, p);
            if (!cic_setup(p, g, i0[k], i1[k], f[k])) {
                atomicOr(status, kStatusMass);
            } else {
                const float mi = m[i];
                if (mi >= 0.f && isfinite(mi) && mi != 0.f) {
                    ok[k] = true;
                    q[k] = ldexp((double)mi, shift);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        lo[d] = min(lo[d], i0[k][d]);
                        hi[d] = max(hi[d], i0[k][d]);
                    }
                }
            }
        }
    }
    // the block's box of lower corners
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
            hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
        }
        if (lane == 0) {
            red[d][w] = lo[d];
            red[3 + d][w] = hi[d];
        }
    }
    __syncthreads();
    int blo[3], dim[3];
    long long vol = 1;
    bool window = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int l = red[d][0], h = red[3 + d][0];
        for (int k = 1; k < kBlock / 64; ++k) {
            l = min(l, red[d][k]);
            h = max(h, red[3 + d][k]);
        }
        blo[d] = l;
        dim[d] = h - l + 2;  // upper corners included; they may lie past the face
        window = window && h >= 0;
        vol *= dim[d] > 0 ? dim[d] : 0;
    }
    window = window && vol > 0 && vol <= kWin;
    if (window) {
        for (int e = threadIdx.x; e < (int)vol; e += kBlock)
            win[e] = 0ull;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kDepPer; ++k) {
            if (!ok[k])
                continue;
            const int bx = i0[k][0] - blo[0], by = i0[k][1] - blo[1], bz = i0[k][2] - blo[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double qab = q[k] * (a ? f[k][0] : 1.0 - f[k][0]) *
                                       (b ? f[k][1] : 1.0 - f[k][1]);
                    const int row = ((bx + a) * dim[1] + (by + b)) * dim[2] + bz;
                    const unsigned long long v0 = (unsigned long long)llrint(qab * (1.0 - f[k][2]));
                    const unsigned long long v1 = (unsigned long long)llrint(qab * f[k][2]);
                    if (v0)
                        atomicAdd(&win[row], v0);
                    if (v1)
                        atomicAdd(&win[row + 1], v1);
                }
        }
        __syncthreads();
        const int plane = dim[1] * dim[2];
        for (int e = threadIdx.x; e < (int)vol; e += kBlock) {
            const unsigned long long v = win[e];
            if (!v)
                continue;
            const int ex = e / plane, r = e - ex * plane, ey = r / dim[2], ez = r - ey * dim[2];
            // window points past the upper face are the periodic images of
            // the first grid plane
            const int gx = blo[0] + ex, gy = blo[1] + ey, gz = blo[2] + ez;
            atomicAdd(acc + ((long long)(gx < g.ng ? gx : gx - g.ng) * g.ng +
                             (gy < g.ng ? gy : gy - g.ng)) * g.ng + (gz < g.ng ? gz : gz - g.ng),
                      v);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kDepPer; ++k) {
        const double wx[2] = {1.0 - f[k][0], f[k][0]}, wy[2] = {1.0 - f[k][1], f[k][1]};
        const double wz0 = 1.0 - f[k][2], wz1 = f[k][2];
        const int ix[2] = {i0[k][0], i1[k][0]}, iy[2] = {i0[k][1], i1[k][1]};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int row = (ix[a] * g.ng + iy[b]) * g.ng;
                const double qab = q[k] * wx[a] * wy[b];
                unsigned long long v0 = ok[k] ? (unsigned long long)llrint(qab * wz0) : 0ull;
                const unsigned long long v1 = ok[k] ? (unsigned long long)llrint(qab * wz1) : 0ull;
                const int k0 = ok[k] ? row + i0[k][2] : -1, k1 = ok[k] ? row + i1[k][2] : -2;
                const int rk = __shfl_up(k1, 1);
                const unsigned long long rv = shfl_up_u64(v1, 1);
                const bool take = lane > 0 && rk == k0;
                if (take)
                    v0 += rv;
                const bool given = __shfl_down((int)take, 1) != 0 && lane < 63;
                if (v0)
                    atomicAdd(acc + k0, v0);
                if (v1 && !given)
                    atomicAdd(acc + k1, v1);
            }
    }
}

// Fixed-point sums -> density (mass / Delta^3) as float32, clearing the
// accumulator for the next call.
__global__ __launch_bounds__(kBlock) void k_pm_density(unsigned long long *__restrict__ acc,
                                                       long long count,
                                                       const unsigned *__restrict__ part,
                                                       int nparts, int n, double inv_vol,
                                                       float *__restrict__ out)
{
    const double unit = ldexp(inv_vol, -fixed_shift(parts_max(part, nparts), n));
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        out[i] = (float)((double)acc[i] * unit);
        acc[i] = 0ull;
    }
}

// ---- FFT ---------------------------------------------------------------
// One block transforms `lines` whole lines of one axis.  Lines of the y and
// x passes are taken consecutive in z, so each row of the block's tile is a
// contiguous run of `lines` complex values in memory.  Two fusions:
//   * the forward z pass may read the fixed-point accumulator directly
//     (converting to density and clearing it);
//   * the x pass may run forward, apply the k-space factors, and run the
//     inverse transform of both output spectra before storing them.

struct FftPass {
    float2 *data[2];   // field of blockIdx.y (plain passes)
    const float2 *tw;
    int ng, log2ng, lines, log2lines;
    int axis;          // 0: x (stride ng^2), 1: y (stride ng), 2: z (stride 1)
    int inverse;
    // forward z pass from the accumulator (acc != nullptr)
    unsigned long long *acc;
    const unsigned *part;
    int nparts, n;
    double inv_vol;
    // fused k space on the x pass (tab != nullptr): data[0] in, data[0] and
    // data[1] out
    const float *tab;
    float g6num, norm;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

__device__ __forceinline__ long long fft_addr(const FftPass &P, long long line, int e)
{
    const int ng = P.ng;
    if (P.axis == 2)
        return (line << P.log2ng) + e;
    const long long hi = line >> P.log2ng, lo = line & (ng - 1);
    if (P.axis == 1)
        return ((hi << P.log2ng) + e) * (long long)ng + lo;
    return ((long long)e << (2 * P.log2ng)) + (hi << P.log2ng) + lo;
}

__device__ __forceinline__ void tile_pos(const FftPass &P, int t, int &j, int &e)
{
    if (P.axis == 2) {
        j = t >> P.log2ng;
        e = t & (P.ng - 1);
    } else {
        j = t & (P.lines - 1);
        e = t >> P.log2lines;
    }
}

// All Stockham stages on ntile (1 or 2) tiles of `lines` rows each, tile t at
// tile + t * tstride, row stride ld.  Radix 2 first when log2 ng is odd, then
// radix 4; natural order in and out.  Every thread of the block must call.
constexpr int kMaxTiles = 2;

__device__ void fft_stages(float2 *tile, int tstride, int ntile, const FftPass &P, int inverse)
{
    const int ng = P.ng, ld = ng + 1, tid = threadIdx.x;
    const int per_tile = P.lines << P.log2ng;
    const float sgn = inverse ? 1.f : -1.f;  // sign of the exponent
    int ns = 1;
    if (P.log2ng & 1) {
        constexpr int kMax = kMaxTiles * kFftElems / 2 / kFftThreads;
        float2 v[kMax][2];
        const int nbt = per_tile >> 1, nb = nbt * ntile, half = ng >> 1;
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int t = bb >= nbt, r = bb - t * nbt;
            const float2 *row = tile + t * tstride + (r >> (P.log2ng - 1)) * ld;
            const int b = r & (half - 1);
            v[c][0] = row[b];
            v[c][1] = row[b + half];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int t = bb >= nbt, r = bb - t * nbt;
            float2 *row = tile + t * tstride + (r >> (P.log2ng - 1)) * ld;
            const int b = r & (half - 1);
            row[2 * b] = cadd(v[c][0], v[c][1]);
            row[2 * b + 1] = csub(v[c][0], v[c][1]);
        }
        __syncthreads();
        ns = 2;
    }
    for (; ns < ng; ns <<= 2) {
        constexpr int kMax = kMaxTiles * kFftElems / 4 / kFftThreads;
        float2 v[kMax][4];
        const int nbt = per_tile >> 2, nb = nbt * ntile, q = ng >> 2, log2q = P.log2ng - 2;
        const int tw_step = ng / (ns * 4);
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int t = bb >= nbt, r = bb - t * nbt;
            const float2 *row = tile + t * tstride + (r >> log2q) * ld;
            const int b = r & (q - 1);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[c][k] = row[b + k * q];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int t = bb >= nbt, r = bb - t * nbt;
            float2 *row = tile + t * tstride + (r >> log2q) * ld;
            const int b = r & (q - 1);
            const int k = b & (ns - 1);
            float2 x0 = v[c][0], x1 = v[c][1], x2 = v[c][2], x3 = v[c][3];
            if (k) {
                const int m = k * tw_step;
                float2 w1 = P.tw[m], w2 = P.tw[2 * m], w3 = P.tw[3 * m];
                if (inverse) {
                    w1.y = -w1.y;
                    w2.y = -w2.y;
                    w3.y = -w3.y;
                }
                x1 = cmul(x1, w1);
                x2 = cmul(x2, w2);
                x3 = cmul(x3, w3);
            }
            const float2 a0 = cadd(x0, x2), a1 = csub(x0, x2);
            const float2 b0 = cadd(x1, x3), d = csub(x1, x3);
            const float2 b1 = make_float2(-sgn * d.y, sgn * d.x);  // d * (sgn i)
            const int o = ((b - k) << 2) + k;
            row[o] = cadd(a0, b0);
            row[o + ns] = cadd(a1, b1);
            row[o + 2 * ns] = csub(a0, b0);
            row[o + 3 * ns] = csub(a1, b1);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kFftThreads) void k_fft_lines(FftPass P)
{
    extern __shared__ float2 tile[];
    const int ng = P.ng, ld = ng + 1;
    const int tot = P.lines << P.log2ng;
    const int tstride = P.lines * ld;
    const long long line0 = (long long)blockIdx.x * P.lines;
    const int tid = threadIdx.x;

    if (P.acc) {  // forward z pass straight from the fixed-point sums
        const double unit = ldexp(P.inv_vol, -fixed_shift(parts_max(P.part, P.nparts), P.n));
        for (int t = tid; t < tot; t += kFftThreads) {
            int j, e;
            tile_pos(P, t, j, e);
            const long long a = fft_addr(P, line0 + j, e);
            tile[j * ld + e] = make_float2((float)((double)P.acc[a] * unit), 0.f);
            P.acc[a] = 0ull;
        }
    } else {
        const float2 *__restrict__ src = P.data[blockIdx.y];
        for (int t = tid; t < tot; t += kFftThreads) {
            int j, e;
            tile_pos(P, t, j, e);
            tile[j * ld + e] = src[fft_addr(P, line0 + j, e)];
        }
    }
    __syncthreads();
    fft_stages(tile, tstride, 1, P, P.inverse);

    if (P.tab) {
        // x pass: row j is the line (y, z) of the spectrum, element e = x.
        // a(k) = -D(k) phi(k), phi = 4 pi G_6 S rho / ng^3; tile 0 receives
        // A_x + i A_y = phi (d_y - i d_x), tile 1 A_z = -i d_z phi.
        const float *e6 = P.tab, *fl = P.tab + ng, *dl = P.tab + 2 * ng;
        for (int t = tid; t < tot; t += kFftThreads) {
            const int j = t >> P.log2ng, x = t & (ng - 1);
            const long long line = line0 + j;
            const int y = (int)(line >> P.log2ng), z = (int)(line & (ng - 1));
            const float den = e6[x] + e6[y] + e6[z];
            const float c = den < 0.f ? P.g6num / den * (fl[x] * fl[y] * fl[z]) * P.norm : 0.f;
            const float2 r = tile[j * ld + x];
            const float px = r.x * c, py = r.y * c;
            const float dx = dl[x], dy = dl[y], dz = dl[z];
            tile[j * ld + x] = make_float2(fmaf(px, dy, py * dx), fmaf(py, dy, -px * dx));
            tile[tstride + j * ld + x] = make_float2(dz * py, -dz * px);
        }
        __syncthreads();
        fft_stages(tile, tstride, 2, P, 1);
        for (int f = 0; f < 2; ++f) {
            float2 *__restrict__ dst = P.data[f];
            for (int t = tid; t < tot; t += kFftThreads) {
                int j, e;
                tile_pos(P, t, j, e);
                dst[fft_addr(P, line0 + j, e)] = tile[f * tstride + j * ld + e];
            }
        }
        return;
    }

    float2 *__restrict__ dst = P.acc ? P.data[0] : P.data[blockIdx.y];
    for (int t = tid; t < tot; t += kFftThreads) {
        int j, e;
        tile_pos(P, t, j, e);
        dst[fft_addr(P, line0 + j, e)] = tile[j * ld + e];
    }
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_pm_interp(Src src, int n, PmGeo g,
                                                      const float2 *__restrict__ ga,
                                                      const float2 *__restrict__ gb,
                                                      float *__restrict__ ax,
                                                      float *__restrict__ ay,
                                                      float *__restrict__ az,
                                                      int *__restrict__ status)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    double p[3], f[3];
    int i0[3], i1[3];
    src.get(i, p);
    float a[3] = {0.f, 0.f, 0.f};
    if (cic_setup(p, g, i0, i1, f)) {
        const double wx[2] = {1.0 - f[0], f[0]}, wy[2] = {1.0 - f[1], f[1]},
                     wz[2] = {1.0 - f[2], f[2]};
        const int ix[2] = {i0[0], i1[0]}, iy[2] = {i0[1], i1[1]}, iz[2] = {i0[2], i1[2]};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const long long row = ((long long)ix[u] * g.ng + iy[v]) * g.ng;
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const float wt = (float)(wx[u] * wy[v] * wz[w]);
                    const float2 xy = ga[row + iz[w]];
                    const float zz = gb[row + iz[w]].x;
                    a[0] = fmaf(wt, xy.x, a[0]);
                    a[1] = fmaf(wt, xy.y, a[1]);
                    a[2] = fmaf(wt, zz, a[2]);
                }
            }
    } else {
        atomicOr(status, kStatusMass);
    }
    ax[i] = a[0];
    ay[i] = a[1];
    az[i] = a[2];
}

// ---- host side ------------------------------------------------------------

constexpr int kMaxParts = 512;  // blocks of the mass maximum

int grid_blocks(long long count)
{
    long long b = (count + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

FftPass fft_pass(const sr_pm *pm, float2 *a, float2 *b, int inverse)
{
    FftPass P{};
    P.data[0] = a;
    P.data[1] = b ? b : a;
    P.tw = pm->tw;
    P.ng = pm->ng;
    P.log2ng = pm->log2ng;
    long long lines = kFftElems / pm->ng;
    const long long nlines = (long long)pm->ng * pm->ng;
    if (lines > nlines)
        lines = nlines;
    P.lines = (int)lines;
    while ((1 << P.log2lines) < P.lines)
        ++P.log2lines;
    P.inverse = inverse;
    return P;
}

int fft_launch(sr_pm *pm, const FftPass &P, int axis, unsigned nfield, int ntile)
{
    FftPass Q = P;
    Q.axis = axis;
    const long long nlines = (long long)pm->ng * pm->ng;
    const size_t lds = (size_t)ntile * P.lines * (pm->ng + 1) * sizeof(float2);
    hipLaunchKernelGGL(k_fft_lines, dim3((unsigned)(nlines / P.lines), nfield),
                       dim3(kFftThreads), lds, pm->ctx->stream, Q);
    return sr_check_launch(pm->ctx, "k_fft_lines");
}

// Plain in-place 3-D transform of one grid.
int fft_enqueue(sr_pm *pm, float2 *a, int inverse)
{
    const FftPass P = fft_pass(pm, a, nullptr, inverse);
    for (int axis = 2; axis >= 0; --axis) {
        int rc = fft_launch(pm, P, axis, 1, 1);
        if (rc)
            return rc;
    }
    return SR_OK;
}

PmGeo pm_geo(const sr_pm *pm)
{
    PmGeo g;
    g.scale = (double)pm->ng / pm->len;
    g.ng = pm->ng;
    g.log2ng = pm->log2ng;
    return g;
}

int parts_for(int n)
{
    int b = (n + kMaxUnroll * kBlock - 1) / (kMaxUnroll * kBlock);
    return b < 1 ? 1 : (b > kMaxParts ? kMaxParts : b);
}

// Mass maximum and the fixed-point deposit into pm->acc; returns the number
// of mass partials written (0 for n == 0).
template <class Src>
int deposit_enqueue(sr_pm *pm, const Src &src, const float *m, int n, int *nparts)
{
    sr_ctx *ctx = pm->ctx;
    *nparts = 0;
    if (n <= 0)
        return SR_OK;
    const int np = parts_for(n);
    hipLaunchKernelGGL(k_pm_mass_max, dim3(np), dim3(kBlock), 0, ctx->stream, m, n, pm->part,
                       ctx->status);
    int rc = sr_check_launch(ctx, "k_pm_mass_max");
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_pm_deposit<Src>, dim3((n + kDepBlock - 1) / kDepBlock), dim3(kBlock), 0,
                       ctx->stream, src, m, n, pm_geo(pm), pm->part, np, pm->acc, ctx->status);
    if ((rc = sr_check_launch(ctx, "k_pm_deposit")))
        return rc;
    *nparts = np;
    return SR_OK;
}

template <class Src>
int force_enqueue_pm(sr_pm *pm, const Src &src, const float *m, int n, float *ax, float *ay,
                     float *az)
{
    sr_ctx *ctx = pm->ctx;
    int np = 0;
    int rc = deposit_enqueue(pm, src, m, n, &np);
    if (rc)
        return rc;
    // forward z (from the accumulator), forward y, then x: forward, k space
    // and inverse of both spectra; inverse y and z on both grids
    FftPass P = fft_pass(pm, pm->ga, pm->gb, 0);
    P.acc = pm->acc;
    P.part = pm->part;
    P.nparts = np;
    P.n = n;
    P.inv_vol = 1.0 / (pm->delta * pm->delta * pm->delta);
    if ((rc = fft_launch(pm, P, 2, 1, 1)))
        return rc;
    P.acc = nullptr;
    if ((rc = fft_launch(pm, P, 1, 1, 1)))
        return rc;
    const long long cells = 1ll << (3 * pm->log2ng);
    P.tab = pm->tab;
    P.g6num = (float)(45.0 / 128.0 * pm->delta * pm->delta);
    P.norm = (float)(4.0 * M_PI / (double)cells);
    if ((rc = fft_launch(pm, P, 0, 1, 2)))
        return rc;
    P.tab = nullptr;
    P.inverse = 1;
    if ((rc = fft_launch(pm, P, 1, 2, 1)) || (rc = fft_launch(pm, P, 2, 2, 1)))
        return rc;
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_pm_interp<Src>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       ctx->stream, src, n, pm_geo(pm), pm->ga, pm->gb, ax, ay, az, ctx->status);
    return sr_check_launch(ctx, "k_pm_interp");
}

int check_pm(sr_pm *pm)
{
    if (!pm || !pm->ctx)
        return SR_EINVAL;
    pm->ctx->err.clear();
    if (hipSetDevice(pm->ctx->device) != hipSuccess)
        return sr_fail(pm->ctx, SR_EDEVICE, "hipSetDevice failed");
    return SR_OK;
}

int check_particles(sr_pm *pm, int64_t n, bool any_null)
{
    if (n < 0 || n > INT_MAX)
        return sr_fail(pm->ctx, SR_EINVAL, "n out of range");
    if (n > 0 && any_null)
        return sr_fail(pm->ctx, SR_EINVAL, "NULL pointer with n > 0");
    return SR_OK;
}

}  // namespace

// Exposed to the step (sr_step.cpp).
int pm_force_split_enqueue(sr_pm *pm, const int32_t *cell3, const float *ox, const float *oy,
                           const float *oz, const float *mass, int n, const double h[3],
                           float *ax, float *ay, float *az)
{
    SrcSplit src{cell3, ox, oy, oz, {h[0], h[1], h[2]}};
    return force_enqueue_pm(pm, src, mass, n, ax, ay, az);
}

sr_ctx *pm_context(const sr_pm *pm) { return pm->ctx; }
double pm_len(const sr_pm *pm) { return pm->len; }

extern "C" int sr_pm_bytes(int32_t ng, size_t *bytes)
{
    if (!bytes || ng < 8 || ng > 1024 || (ng & (ng - 1)))
        return SR_EINVAL;
    const size_t cells = (size_t)ng * ng * ng;
    *bytes = 2 * cells * sizeof(float2) + cells * sizeof(unsigned long long) +
             (size_t)ng * sizeof(float2) + 3 * (size_t)ng * sizeof(float) +
             kMaxParts * sizeof(unsigned);
    return SR_OK;
}

extern "C" int sr_pm_create(sr_ctx *ctx, int32_t ng, double len, float sigma, int32_t ns,
                            sr_pm **out)
{
    if (!ctx || !out)
        return SR_EINVAL;
    ctx->err.clear();
    *out = nullptr;
    if (ng < 8 || ng > 1024 || (ng & (ng - 1)))
        return sr_fail(ctx, SR_EINVAL, "ng must be a power of two in [8, 1024]");
    if (!(len > 0.0) || !std::isfinite(len))
        return sr_fail(ctx, SR_EINVAL, "len must be positive and finite");
    if (!(sigma > 0.f) || !std::isfinite(sigma) || ns < 0 || ns > 16)
        return sr_fail(ctx, SR_EINVAL, "filter needs sigma > 0 and 0 <= ns <= 16");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    sr_pm *pm = new sr_pm;
    pm->ctx = ctx;
    pm->ng = ng;
    while ((1 << pm->log2ng) < ng)
        ++pm->log2ng;
    pm->len = len;
    pm->delta = len / ng;
    pm->sigma = sigma;
    pm->ns = ns;
    const size_t cells = (size_t)ng * ng * ng;
    bool ok = hipMalloc(&pm->ga, cells * sizeof(float2)) == hipSuccess &&
              hipMalloc(&pm->gb, cells * sizeof(float2)) == hipSuccess &&
              hipMalloc(&pm->tw, ng * sizeof(float2)) == hipSuccess &&
              hipMalloc(&pm->tab, 3 * ng * sizeof(float)) == hipSuccess &&
              hipMalloc(&pm->acc, cells * sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&pm->part, kMaxParts * sizeof(unsigned)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        sr_pm_destroy(pm);
        return sr_fail(ctx, SR_ENOMEM, "PM grids: device allocation failed");
    }
    // Tables in FP64, rounded once.  Frequency index n stands for the signed
    // integer frequency nn (n >= ng/2 -> n - ng), k = 2 pi nn / len.
    std::vector<float2> tw(ng);
    std::vector<float> tab(3 * ng);
    const double d = pm->delta, sd = (double)sigma * d;
    for (int m = 0; m < ng; ++m) {
        const double a = -2.0 * M_PI * m / ng;
        tw[m] = make_float2((float)cos(a), (float)sin(a));
    }
    for (int n = 0; n < ng; ++n) {
        const int nn = n < ng / 2 ? n : n - ng;
        const double k = 2.0 * M_PI * nn / len, h = k * d;
        // G_6 axis term minus its k = 0 value 945/1024, exactly 0 at k = 0
        const double e6 = nn == 0 ? 0.0
                                  : (cos(h) - 1.0) - 5.0 / 64.0 * (cos(2 * h) - 1.0) +
                                        1.0 / 1024.0 * (cos(4 * h) - 1.0);
        const double x = 0.5 * h;
        const double sinc = nn == 0 ? 1.0 : sin(x) / x;
        tab[n] = (float)e6;
        tab[ng + n] = (float)(exp(-k * k * sd * sd / 4.0) * pow(sinc, ns));
        tab[2 * ng + n] = (float)((4.0 / 3.0 * sin(h) - 1.0 / 6.0 * sin(2 * h)) / d);
    }
    if (hipMemset(pm->acc, 0, cells * sizeof(unsigned long long)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(pm->tw, tw.data(), ng * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pm->tab, tab.data(), 3 * ng * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess) {
        sr_pm_destroy(pm);
        return sr_fail(ctx, SR_EDEVICE, "PM table upload failed");
    }
    *out = pm;
    return SR_OK;
}

extern "C" int sr_pm_destroy(sr_pm *pm)
{
    if (!pm)
        return SR_EINVAL;
    if (pm->ctx) {
        (void)hipSetDevice(pm->ctx->device);
        (void)hipStreamSynchronize(pm->ctx->stream);
    }
    (void)hipFree(pm->ga);
    (void)hipFree(pm->gb);
    (void)hipFree(pm->tw);
    (void)hipFree(pm->tab);
    (void)hipFree(pm->acc);
    (void)hipFree(pm->part);
    delete pm;
    return SR_OK;
}

extern "C" int sr_pm_deposit(sr_pm *pm, const float *x, const float *y, const float *z,
                             const float *mass, int64_t n, float *rho)
{
    int rc = check_pm(pm);
    if (rc)
        return rc;
    if ((rc = check_particles(pm, n, !x || !y || !z || !mass)))
        return rc;
    if (!rho)
        return sr_fail(pm->ctx, SR_EINVAL, "rho is NULL");
    int np = 0;
    if ((rc = deposit_enqueue(pm, SrcGlobal{x, y, z}, mass, (int)n, &np)))
        return rc;
    const long long cells = 1ll << (3 * pm->log2ng);
    hipLaunchKernelGGL(k_pm_density, dim3(grid_blocks(cells)), dim3(kBlock), 0,
                       pm->ctx->stream, pm->acc, cells, pm->part, np, (int)n,
                       1.0 / (pm->delta * pm->delta * pm->delta), rho);
    return sr_check_launch(pm->ctx, "k_pm_density");
}

extern "C" int sr_pm_fft(sr_pm *pm, float *data, int32_t inverse)
{
    int rc = check_pm(pm);
    if (rc)
        return rc;
    if (!data)
        return sr_fail(pm->ctx, SR_EINVAL, "data is NULL");
    return fft_enqueue(pm, reinterpret_cast<float2 *>(data), inverse ? 1 : 0);
}

extern "C" int sr_pm_force(sr_pm *pm, const float *x, const float *y, const float *z,
                           const float *mass, int64_t n, float *ax, float *ay, float *az)
{
    int rc = check_pm(pm);
    if (rc)
        return rc;
    if ((rc = check_particles(pm, n, !x || !y || !z || !mass || !ax || !ay || !az)))
        return rc;
    return force_enqueue_pm(pm, SrcGlobal{x, y, z}, mass, (int)n, ax, ay, az);
}

extern "C" int sr_pm_force_split(sr_pm *pm, const int32_t *cell3, const float *ox,
                                 const float *oy, const float *oz, const float *mass, int64_t n,
                                 double cell, float *ax, float *ay, float *az)
{
    int rc = check_pm(pm);
    if (rc)
        return rc;
    if ((rc = check_particles(pm, n, !cell3 || !ox || !oy || !oz || !mass || !ax || !ay || !az)))
        return rc;
    sr_box box;
    box.len[0] = box.len[1] = box.len[2] = pm->len;
    box.periodic = 1;
    box._pad = 0;
    box.skin = 0.0;
    SplitGeom sg;
    if ((rc = split_geom(pm->ctx, &box, cell, &sg)))
        return rc;
    return pm_force_split_enqueue(pm, cell3, ox, oy, oz, mass, (int)n, sg.h, ax, ay, az);
}
