// Long-range particle-mesh force (Sec. 2.3) on one GPU.
//
//   deposit   CIC weights from FP64 grid coordinates; every particle adds its
//             8 contributions to a 64-bit fixed-point grid with integer
//             atomics, so the density is independent of arrival order.
//   FFT       radix-4 (and one radix-2) Stockham passes in LDS along z, y
//             and x; the twiddles are an FP64-built float32 table.
//   k space   one kernel applies 4 pi G_6 S (Eqs. (greenf), (filter)) and
//             the Super-Lanczos gradient (Eq. (sldiff)), writing two spectra:
//             A_x + i A_y and A_z.  Each A_d is the transform of a real field,
//             so one complex inverse FFT returns a_x and a_y together.
//   interp    CIC gather of (a_x, a_y, a_z) at each particle.
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
    float2 *gb = nullptr;   // complex grid; 64-bit deposit accumulator, then A_z
    float2 *tw = nullptr;   // [ng] exp(-2 pi i m / ng)
    float *tab = nullptr;   // [3 ng] G_6 axis term, filter factor, gradient factor
    unsigned *mmax = nullptr;  // [1] bit pattern of the largest mass
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

__global__ __launch_bounds__(kBlock) void k_pm_clear(unsigned long long *__restrict__ acc,
                                                     long long count, unsigned *__restrict__ mmax)
{
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride)
        acc[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *mmax = 0u;
}

// Largest mass (bit pattern of a non-negative float orders like the value);
// a negative or non-finite mass sets the status.
__global__ __launch_bounds__(kBlock) void k_pm_mass_max(const float *__restrict__ m, int n,
                                                        unsigned *__restrict__ mmax,
                                                        int *__restrict__ status)
{
    __shared__ unsigned part[kBlock / 64];
    unsigned v = 0u;
    bool bad = false;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const float mi = m[i];
        if (!(mi >= 0.f) || !isfinite(mi))
            bad = true;
        else
            v = max(v, __float_as_uint(mi));
    }
    if (bad)
        atomicOr(status, kStatusMass);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = max(v, (unsigned)__shfl_xor((int)v, off));
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned b = part[0];
        for (int w = 1; w < kBlock / 64; ++w)
            b = max(b, part[w]);
        atomicMax(mmax, b);
    }
}

template <class Src>
__global__ __launch_bounds__(kBlock) void k_pm_deposit(Src src, const float *__restrict__ m, int n,
                                                       PmGeo g, const unsigned *__restrict__ mmax,
                                                       unsigned long long *__restrict__ acc,
                                                       int *__restrict__ status)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    double p[3], f[3];
    int i0[3], i1[3];
    src.get(i, p);
    if (!cic_setup(p, g, i0, i1, f)) {
        atomicOr(status, kStatusMass);
        return;
    }
    const float mi = m[i];
    if (!(mi >= 0.f) || !isfinite(mi) || mi == 0.f)
        return;
    const double q = ldexp((double)mi, fixed_shift(*mmax, n));
    const double wx[2] = {1.0 - f[0], f[0]}, wy[2] = {1.0 - f[1], f[1]},
                 wz[2] = {1.0 - f[2], f[2]};
    const int ix[2] = {i0[0], i1[0]}, iy[2] = {i0[1], i1[1]}, iz[2] = {i0[2], i1[2]};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double qab = q * wx[a] * wy[b];
            const long long row = ((long long)ix[a] * g.ng + iy[b]) * g.ng;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const unsigned long long v = (unsigned long long)llrint(qab * wz[c]);
                if (v)
                    atomicAdd(acc + row + iz[c], v);
            }
        }
}

// Fixed-point sums -> density (mass / Delta^3): complex (rho, 0) into a grid
// or plain float32 into an output array.
__global__ __launch_bounds__(kBlock) void k_pm_density(const unsigned long long *__restrict__ acc,
                                                       long long count,
                                                       const unsigned *__restrict__ mmax, int n,
                                                       double inv_vol, float2 *__restrict__ outc,
                                                       float *__restrict__ outr)
{
    const double unit = ldexp(inv_vol, -fixed_shift(*mmax, n));
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const float r = (float)((double)acc[i] * unit);
        if (outc)
            outc[i] = make_float2(r, 0.f);
        else
            outr[i] = r;
    }
}

// ---- FFT ---------------------------------------------------------------
// One block transforms `lines` whole lines of one axis.  Lines of the y and
// x passes are taken consecutive in z, so each row of the block's tile is a
// contiguous run of `lines` complex values in memory.

struct FftPass {
    float2 *data[2];
    const float2 *tw;
    int ng, log2ng, lines, log2lines;
    int axis;      // 0: x (stride ng^2), 1: y (stride ng), 2: z (stride 1)
    int inverse;
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

__global__ __launch_bounds__(kFftThreads) void k_fft_lines(FftPass P)
{
    extern __shared__ float2 tile[];
    float2 *__restrict__ data = P.data[blockIdx.y];
    const int ng = P.ng, ld = ng + 1;
    const int tot = P.lines << P.log2ng;
    const long long line0 = (long long)blockIdx.x * P.lines;
    const int tid = threadIdx.x;
    for (int t = tid; t < tot; t += kFftThreads) {
        int j, e;
        if (P.axis == 2) {
            j = t >> P.log2ng;
            e = t & (ng - 1);
        } else {
            j = t & (P.lines - 1);
            e = t >> P.log2lines;
        }
        tile[j * ld + e] = data[fft_addr(P, line0 + j, e)];
    }
    __syncthreads();

    const float sgn = P.inverse ? 1.f : -1.f;  // sign of the exponent
    int ns = 1;
    if (P.log2ng & 1) {  // one radix-2 stage (ns = 1: no twiddles)
        constexpr int kMax = kFftElems / 2 / kFftThreads;
        float2 v[kMax][2];
        const int nb = tot >> 1, half = ng >> 1;
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int j = bb >> (P.log2ng - 1), b = bb & (half - 1);
            v[c][0] = tile[j * ld + b];
            v[c][1] = tile[j * ld + b + half];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int j = bb >> (P.log2ng - 1), b = bb & (half - 1);
            tile[j * ld + 2 * b] = cadd(v[c][0], v[c][1]);
            tile[j * ld + 2 * b + 1] = csub(v[c][0], v[c][1]);
        }
        __syncthreads();
        ns = 2;
    }
    for (; ns < ng; ns <<= 2) {
        constexpr int kMax = kFftElems / 4 / kFftThreads;
        float2 v[kMax][4];
        const int nb = tot >> 2, q = ng >> 2, log2q = P.log2ng - 2;
        const int tw_step = ng / (ns * 4);
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int j = bb >> log2q, b = bb & (q - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[c][r] = tile[j * ld + b + r * q];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kMax; ++c) {
            const int bb = tid + c * kFftThreads;
            if (bb >= nb)
                break;
            const int j = bb >> log2q, b = bb & (q - 1);
            const int k = b & (ns - 1);
            float2 x0 = v[c][0], x1 = v[c][1], x2 = v[c][2], x3 = v[c][3];
            if (k) {
                const int m = k * tw_step;
                float2 w1 = P.tw[m], w2 = P.tw[2 * m], w3 = P.tw[3 * m];
                if (P.inverse) {
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
            float2 *row = tile + j * ld;
            row[o] = cadd(a0, b0);
            row[o + ns] = cadd(a1, b1);
            row[o + 2 * ns] = csub(a0, b0);
            row[o + 3 * ns] = csub(a1, b1);
        }
        __syncthreads();
    }

    for (int t = tid; t < tot; t += kFftThreads) {
        int j, e;
        if (P.axis == 2) {
            j = t >> P.log2ng;
            e = t & (ng - 1);
        } else {
            j = t & (P.lines - 1);
            e = t >> P.log2lines;
        }
        data[fft_addr(P, line0 + j, e)] = tile[j * ld + e];
    }
}

// rho(k) -> A_x + i A_y (in place) and A_z: a(k) = -D(k) phi(k),
// phi = 4 pi G_6 S rho / ng^3 (the inverse transforms are unnormalised).
__global__ __launch_bounds__(kBlock) void k_pm_kspace(float2 *__restrict__ ga,
                                                      float2 *__restrict__ gb,
                                                      const float *__restrict__ tab, int ng,
                                                      int log2ng, float g6num, float norm)
{
    const long long total = 1ll << (3 * log2ng);
    const long long stride = (long long)gridDim.x * kBlock;
    const float *e6 = tab, *fl = tab + ng, *dl = tab + 2 * ng;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total; i += stride) {
        const int z = (int)(i & (ng - 1)), y = (int)((i >> log2ng) & (ng - 1)),
                  x = (int)(i >> (2 * log2ng));
        const float den = e6[x] + e6[y] + e6[z];
        const float c = den < 0.f ? g6num / den * (fl[x] * fl[y] * fl[z]) * norm : 0.f;
        const float2 r = ga[i];
        const float px = r.x * c, py = r.y * c;  // phi
        const float dx = dl[x], dy = dl[y], dz = dl[z];
        ga[i] = make_float2(fmaf(px, dy, py * dx), fmaf(py, dy, -px * dx));
        gb[i] = make_float2(dz * py, -dz * px);
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

int grid_blocks(long long count)
{
    long long b = (count + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

int fft_enqueue(sr_pm *pm, float2 *a, float2 *b, int inverse)
{
    sr_ctx *ctx = pm->ctx;
    FftPass P;
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
    P.log2lines = 0;
    while ((1 << P.log2lines) < P.lines)
        ++P.log2lines;
    P.inverse = inverse;
    const size_t lds = (size_t)P.lines * (pm->ng + 1) * sizeof(float2);
    const dim3 grid((unsigned)(nlines / lines), b ? 2u : 1u);
    for (int axis = 2; axis >= 0; --axis) {
        P.axis = axis;
        hipLaunchKernelGGL(k_fft_lines, grid, dim3(kFftThreads), lds, ctx->stream, P);
        int rc = sr_check_launch(ctx, "k_fft_lines");
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

template <class Src>
int deposit_enqueue(sr_pm *pm, const Src &src, const float *m, int n, float *rho_out)
{
    sr_ctx *ctx = pm->ctx;
    const long long cells = 1ll << (3 * pm->log2ng);
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(pm->gb);
    hipLaunchKernelGGL(k_pm_clear, dim3(grid_blocks(cells)), dim3(kBlock), 0, ctx->stream, acc,
                       cells, pm->mmax);
    int rc = sr_check_launch(ctx, "k_pm_clear");
    if (rc)
        return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_pm_mass_max, dim3(grid_blocks(n) < 1024 ? grid_blocks(n) : 1024),
                           dim3(kBlock), 0, ctx->stream, m, n, pm->mmax, ctx->status);
        if ((rc = sr_check_launch(ctx, "k_pm_mass_max")))
            return rc;
        hipLaunchKernelGGL(k_pm_deposit<Src>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                           ctx->stream, src, m, n, pm_geo(pm), pm->mmax, acc, ctx->status);
        if ((rc = sr_check_launch(ctx, "k_pm_deposit")))
            return rc;
    }
    const double inv_vol = 1.0 / (pm->delta * pm->delta * pm->delta);
    hipLaunchKernelGGL(k_pm_density, dim3(grid_blocks(cells)), dim3(kBlock), 0, ctx->stream, acc,
                       cells, pm->mmax, n, inv_vol, rho_out ? nullptr : pm->ga, rho_out);
    return sr_check_launch(ctx, "k_pm_density");
}

template <class Src>
int force_enqueue_pm(sr_pm *pm, const Src &src, const float *m, int n, float *ax, float *ay,
                     float *az)
{
    sr_ctx *ctx = pm->ctx;
    int rc = deposit_enqueue(pm, src, m, n, nullptr);
    if (rc)
        return rc;
    if ((rc = fft_enqueue(pm, pm->ga, nullptr, 0)))
        return rc;
    const long long cells = 1ll << (3 * pm->log2ng);
    const float g6num = (float)(45.0 / 128.0 * pm->delta * pm->delta);
    const float norm = (float)(4.0 * M_PI / (double)cells);
    hipLaunchKernelGGL(k_pm_kspace, dim3(grid_blocks(cells)), dim3(kBlock), 0, ctx->stream, pm->ga,
                       pm->gb, pm->tab, pm->ng, pm->log2ng, g6num, norm);
    if ((rc = sr_check_launch(ctx, "k_pm_kspace")))
        return rc;
    if ((rc = fft_enqueue(pm, pm->ga, pm->gb, 1)))
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
    *bytes = 2 * cells * sizeof(float2) + (size_t)ng * sizeof(float2) + 3 * (size_t)ng * sizeof(float) +
             256;
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
              hipMalloc(&pm->mmax, sizeof(unsigned)) == hipSuccess;
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
    if (hipMemcpy(pm->tw, tw.data(), ng * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
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
    (void)hipFree(pm->mmax);
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
    return deposit_enqueue(pm, SrcGlobal{x, y, z}, mass, (int)n, rho);
}

extern "C" int sr_pm_fft(sr_pm *pm, float *data, int32_t inverse)
{
    int rc = check_pm(pm);
    if (rc)
        return rc;
    if (!data)
        return sr_fail(pm->ctx, SR_EINVAL, "data is NULL");
    return fft_enqueue(pm, reinterpret_cast<float2 *>(data), nullptr, inverse ? 1 : 0);
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
