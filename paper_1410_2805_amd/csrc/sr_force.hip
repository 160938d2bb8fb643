// Short-range particle-particle force on gfx950 (Eq. (force), Sec. 3.1).
//
// After binning (sr_bin.hip) the particles sit cell by cell in a float4
// (x, y, z, m) copy.  Each force work item is one cell's chunk of at most 64
// targets.  One wavefront owns an item:
//   - the 27 neighbour cells are 9 rows of 3 cells that are contiguous in the
//     sorted order, so the source list is at most 18 contiguous pieces (a row
//     splits in two where it wraps around a periodic face);
//   - sources are staged through LDS in tiles of kTile with their periodic
//     image shift applied, then read back by broadcast;
//   - when a cell holds few targets the 64 lanes are split into S groups that
//     take every S-th source of a tile, and the groups' sums are added by
//     cross-lane shuffles at the end;
//   - the pair loop is plain float32 VALU: one reciprocal square root,
//     the polynomial in registers, the cutoff as a select (Sec. 3.1 describes
//     the same select-based filtering inside the force loop).
// Periodic images are made exact: a target in the last cell layer of an axis
// works in a frame shifted by -L there, so every image shift is 0 or -L and is
// only ever applied to coordinates >= L/2, where subtracting L is exact.
#include <climits>
#include <cmath>

#include "sr_internal.h"

namespace {

constexpr int kTile = 256;       // sources per LDS tile (4 KiB)
constexpr float kFar = 1.0e6f;   // padding source far outside any box, mass 0

struct Stencil {
    int pbeg[19];      // prefix of piece lengths; pbeg[18] = all sources
    int psrc[18];      // first sorted slot of each piece
    float4 psh[18];    // image shift of each piece
};

__device__ __forceinline__ int wave_exclusive_scan(int v, int lane, int *total)
{
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += t;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

// Builds the source pieces of target cell (cx, cy, cz) into st (all lanes
// call; lanes < 18 each own one piece slot: row r = lane/2, half = lane%2).
__device__ void build_stencil(Stencil &st, const int *__restrict__ offsets, const Geom &g, int cx,
                              int cy, int cz, const float F[3], int lane)
{
    int len = 0, src = 0;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (lane < 18) {
        const int r = lane >> 1, half = lane & 1;
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        int ny = cy + dy, nz = cz + dz;
        float shy = F[1], shz = F[2];
        bool ok = true;
        if (g.periodic) {
            if (ny < 0) { ny += g.nc[1]; shy -= g.lenf[1]; }
            else if (ny >= g.nc[1]) { ny -= g.nc[1]; shy += g.lenf[1]; }
            if (nz < 0) { nz += g.nc[2]; shz -= g.lenf[2]; }
            else if (nz >= g.nc[2]) { nz -= g.nc[2]; shz += g.lenf[2]; }
        } else {
            ok = ny >= 0 && ny < g.nc[1] && nz >= 0 && nz < g.nc[2];
        }
        int x0 = 0, x1 = -1;
        float shx = F[0];
        const int n0 = g.nc[0];
        const int lo = cx - g.hx, hi = cx + g.hx;
        if (ok) {
            if (g.periodic) {
                if (lo < 0) {
                    if (half == 0) { x0 = 0; x1 = hi; }
                    else { x0 = lo + n0; x1 = n0 - 1; shx -= g.lenf[0]; }
                } else if (hi >= n0) {
                    if (half == 0) { x0 = lo; x1 = n0 - 1; }
                    else { x0 = 0; x1 = hi - n0; shx += g.lenf[0]; }
                } else if (half == 0) {
                    x0 = lo;
                    x1 = hi;
                }
            } else if (half == 0) {
                x0 = lo > 0 ? lo : 0;
                x1 = hi < n0 - 1 ? hi : n0 - 1;
            }
        }
        if (x1 >= x0) {
            const int row = n0 * (ny + g.nc[1] * nz);
            src = offsets[row + x0];
            len = offsets[row + x1 + 1] - src;
        }
        sx = shx;
        sy = shy;
        sz = shz;
    }
    int total;
    int beg = wave_exclusive_scan(len, lane, &total);
    if (lane < 18) {
        st.pbeg[lane] = beg;
        st.psrc[lane] = src;
        st.psh[lane] = make_float4(sx, sy, sz, 0.f);
    }
    if (lane == 0)
        st.pbeg[18] = total;
}

// A target whose stencil wraps past the upper face of an axis works in a
// frame shifted by -L along it: its coordinate and the unwrapped sources are
// all >= L/2 there, so subtracting L is exact, and the wrapped sources need
// no shift at all.
__device__ __forceinline__ void frame_shift(const Geom &g, const int cc[3], float F[3])
{
    const int h[3] = {g.hx, 1, 1};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        F[d] = (g.periodic && cc[d] + h[d] >= g.nc[d]) ? -g.lenf[d] : 0.f;
}

__device__ __forceinline__ void decode_cell(int cell, const Geom &g, int &cx, int &cy, int &cz)
{
    const int plane = g.nc[0] * g.nc[1];
    cz = cell / plane;
    const int rem = cell - cz * plane;
    cy = rem / g.nc[0];
    cx = rem - cy * g.nc[0];
}

__device__ __forceinline__ bool is_passive(float4 p, const Geom &g)
{
    if (g.periodic)
        return false;
    const double c[3] = {(double)p.x, (double)p.y, (double)p.z};
    bool pas = false;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        pas = pas || (c[d] < g.skin) || (g.len[d] - c[d] < g.skin);
    return pas;
}

// Stage sources [g0, g0 + cntp) of the stencil into the tile.
__device__ __forceinline__ void stage_tile(float4 *tile, const Stencil &st,
                                           const float4 *__restrict__ sorted, int g0, int cnt,
                                           int cntp, int lane, int &p)
{
    for (int q = lane; q < cntp; q += 64) {
        float4 v = make_float4(kFar, kFar, kFar, 0.f);
        if (q < cnt) {
            const int gi = g0 + q;
            while (gi >= st.pbeg[p + 1])
                ++p;
            const float4 s = sorted[st.psrc[p] + (gi - st.pbeg[p])];
            const float4 sh = st.psh[p];
            v = make_float4(s.x + sh.x, s.y + sh.y, s.z + sh.z, s.w);
        }
        tile[q] = v;
    }
}

// One tile of pair interactions for one lane: sources src[0 .. cnt) (cnt a
// multiple of 4), target (xi, yi, zi); partial sums into tx, ty, tz.
template <bool kUniformMass>
__device__ __forceinline__ void pair_tile(const float4 *src, int cnt, float xi, float yi, float zi,
                                          const ForceParams &fp, float &tx, float &ty, float &tz)
{
    const float eps = fp.eps, rcut = fp.rcut, q0 = fp.q0;
    const float n1 = fp.nq[1], n2 = fp.nq[2], n3 = fp.nq[3], n4 = fp.nq[4], n5 = fp.nq[5];
    for (int j = 0; j < cnt; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float4 s = src[j + u];
            const float dx = s.x - xi;
            const float dy = s.y - yi;
            const float dz = s.z - zi;
            // se = s + eps; f = se^(-3/2) - q(se) with q(se) = p(se - eps)
            const float se = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps)));
            const float rs = __builtin_amdgcn_rsqf(se);
            const float rs2 = rs * rs;
            const float tt = fmaf(rs2, rs, -q0);
            float h = fmaf(n5, se, n4);
            h = fmaf(h, se, n3);
            h = fmaf(h, se, n2);
            h = fmaf(h, se, n1);
            float f = fmaf(h, se, tt);
            f = se < rcut ? f : 0.f;  // cutoff by select: also zeroes padding
            if (!kUniformMass)
                f *= s.w;
            tx = fmaf(f, dx, tx);
            ty = fmaf(f, dy, ty);
            tz = fmaf(f, dz, tz);
        }
    }
}

// One wavefront per work item (a chunk of nt <= 64 targets of one cell).
// Lane L serves target t = L mod nt in group part = L / nt; the S groups
// split each staged tile into S contiguous slices.
__global__ __launch_bounds__(64) void k_force(const int4 *__restrict__ items,
                                              const int *__restrict__ n_items,
                                              const float4 *__restrict__ sorted,
                                              const int *__restrict__ offsets,
                                              const int *__restrict__ perm,
                                              const int *__restrict__ mass_mixed, Geom g,
                                              ForceParams fp, float *__restrict__ ax,
                                              float *__restrict__ ay, float *__restrict__ az)
{
    __shared__ float4 tile[kTile + 4 * kMaxSplit];
    __shared__ Stencil st;
    const int lane = threadIdx.x;
    // Workgroups are dealt to the 8 XCDs round-robin; give XCD k the k-th
    // contiguous eighth of the items so that neighbouring cells, which share
    // most of their sources, meet in the same L2.
    const int nitems = *n_items;
    const int per = (nitems + 7) >> 3;
    const int it = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || it >= nitems)
        return;
    const int4 item = items[it];
    const int cell = item.x, kb = item.y, nt = item.z, S = item.w;
    int cx, cy, cz;
    decode_cell(cell, g, cx, cy, cz);
    const int cc[3] = {cx, cy, cz};
    float F[3];
    frame_shift(g, cc, F);
    build_stencil(st, offsets, g, cx, cy, cz, F, lane);

    const int part = lane / nt;
    const int t = lane - part * nt;
    const bool has_target = part < S;
    const float4 pt = sorted[kb + t];
    const bool pas = is_passive(pt, g);
    const float xi = pt.x + F[0], yi = pt.y + F[1], zi = pt.z + F[2];
    const bool uniform = *mass_mixed == 0;
    __syncthreads();

    float acx = 0.f, acy = 0.f, acz = 0.f;
    if (__any(has_target && !pas)) {
        const int total = st.pbeg[18];
        const int quantum = 4 * S;
        int p = 0;
        for (int g0 = 0; g0 < total; g0 += kTile) {
            const int cnt = total - g0 < kTile ? total - g0 : kTile;
            const int cntp = (cnt + quantum - 1) / quantum * quantum;
            stage_tile(tile, st, sorted, g0, cnt, cntp, lane, p);
            __syncthreads();
            const int slice = cntp / S;
            const float4 *src = tile + (has_target ? part : 0) * slice;
            float tx = 0.f, ty = 0.f, tz = 0.f;
            if (uniform)
                pair_tile<true>(src, slice, xi, yi, zi, fp, tx, ty, tz);
            else
                pair_tile<false>(src, slice, xi, yi, zi, fp, tx, ty, tz);
            acx += tx;
            acy += ty;
            acz += tz;
            __syncthreads();
        }
        if (uniform) {
            acx *= pt.w;
            acy *= pt.w;
            acz *= pt.w;
        }
    }
    // add the S group sums of each target in group order
    float4 *red = tile;
    red[lane] = make_float4(acx, acy, acz, 0.f);
    __syncthreads();
    if (part == 0) {
        for (int q = 1; q < S; ++q) {
            const float4 o = red[t + q * nt];
            acx += o.x;
            acy += o.y;
            acz += o.z;
        }
        const int orig = perm[kb + t];
        ax[orig] = pas ? 0.f : acx;
        ay[orig] = pas ? 0.f : acy;
        az[orig] = pas ? 0.f : acz;
    }
}

// Useful-pair and candidate counts with the same stencil and cutoff test.
__global__ __launch_bounds__(64) void k_pair_stats(const int4 *__restrict__ items,
                                                   const int *__restrict__ n_items,
                                                   const float4 *__restrict__ sorted,
                                                   const int *__restrict__ offsets,
                                                   const int *__restrict__ perm, Geom g,
                                                   ForceParams fp, int *__restrict__ per_target,
                                                   unsigned long long *__restrict__ stats)
{
    __shared__ float4 tile[kTile];
    __shared__ Stencil st;
    const int lane = threadIdx.x;
    const int it = blockIdx.x;
    if (it >= *n_items)
        return;
    const int4 item = items[it];
    const int cell = item.x, kb = item.y, nt = item.z;
    int cx, cy, cz;
    decode_cell(cell, g, cx, cy, cz);
    const int cc[3] = {cx, cy, cz};
    float F[3];
    frame_shift(g, cc, F);
    build_stencil(st, offsets, g, cx, cy, cz, F, lane);
    const bool has_target = lane < nt;
    const float4 pt = sorted[kb + (has_target ? lane : 0)];
    const bool pas = is_passive(pt, g);
    const bool act = has_target && !pas;
    const float xi = pt.x + F[0], yi = pt.y + F[1], zi = pt.z + F[2];
    __syncthreads();
    const int total = st.pbeg[18];
    int cntu = 0;
    int p = 0;
    for (int g0 = 0; g0 < total; g0 += kTile) {
        const int cnt = total - g0 < kTile ? total - g0 : kTile;
        const int cntp = (cnt + 63) & ~63;
        stage_tile(tile, st, sorted, g0, cnt, cntp, lane, p);
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const float4 s = tile[j];
            const float dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
            const float se = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, fp.eps)));
            cntu += se < fp.rcut ? 1 : 0;
        }
        __syncthreads();
    }
    cntu = act ? cntu - 1 : 0;  // the target itself is always in its stencil
    if (has_target && per_target)
        per_target[perm[kb + lane]] = cntu;
    unsigned long long u = (unsigned long long)cntu;
    unsigned long long c = act ? (unsigned long long)total : 0ull;
    for (int o = 1; o < 64; o <<= 1) {
        u += __shfl_xor(u, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if (lane == 0) {
        atomicAdd(&stats[0], u);
        atomicAdd(&stats[1], c);
    }
}

// One thread per cell: the cell's targets split into chunk_count[c] nearly
// equal chunks of at most kChunk.
__global__ void k_items(const int *__restrict__ offsets, const int *__restrict__ item_off,
                        int ncell, int4 *__restrict__ items)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell)
        return;
    const int b = offsets[c];
    const int len = offsets[c + 1] - b;
    const int q = item_off[c + 1] - item_off[c];
    for (int k = 0; k < q; ++k) {
        const int lo = (int)((long long)k * len / q);
        const int hi = (int)((long long)(k + 1) * len / q);
        items[item_off[c] + k] = make_int4(c, b + lo, hi - lo, split_for(hi - lo));
    }
}

constexpr int kRedBlocks = 256;

// FP64 sum_i m_i a_i: fixed per-thread ranges, fixed tree order.
__global__ __launch_bounds__(256) void k_momentum_partial(const float *__restrict__ m,
                                                          const float *__restrict__ ax,
                                                          const float *__restrict__ ay,
                                                          const float *__restrict__ az, int n,
                                                          double *__restrict__ part)
{
    __shared__ double sh[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += kRedBlocks * 256) {
        const double mi = (double)m[i];
        s[0] += mi * (double)ax[i];
        s[1] += mi * (double)ay[i];
        s[2] += mi * (double)az[i];
    }
    for (int d = 0; d < 3; ++d)
        sh[d][threadIdx.x] = s[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int d = 0; d < 3; ++d)
                sh[d][threadIdx.x] += sh[d][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d)
            part[3 * blockIdx.x + d] = sh[d][0];
}

__global__ void k_momentum_final(const double *__restrict__ part, double *__restrict__ out)
{
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int b = 0; b < kRedBlocks; ++b)
            s += part[3 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

struct ForceScratch {
    BinScratch bin;
    int *offsets;
    int *perm;
    float4 *sorted;
    int *chunk_count;
    int *item_off;    // [ncell + 1]; item_off[ncell] = number of items
    int *scan_part2;
    int4 *items;
    double *mom_part;
};

int64_t item_bound(int64_t n, int ncell)
{
    int64_t nonempty = n < ncell ? n : ncell;
    return nonempty + n / 16 + 1;  // see chunks_for
}

void force_layout(Bump &b, int64_t n, const Geom &g, ForceScratch &s)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    bin_layout(b, n, g, s.bin);
    s.offsets = b.take<int>((size_t)g.ncell + 1);
    s.perm = b.take<int>(nn);
    s.sorted = b.take<float4>(nn);
    s.chunk_count = b.take<int>((size_t)g.ncell);
    s.item_off = b.take<int>((size_t)g.ncell + 1);
    scan_layout(b, g.ncell, &s.scan_part2);
    s.items = b.take<int4>((size_t)item_bound(n, g.ncell));
    s.mom_part = b.take<double>(3 * kRedBlocks);
}

int check_force_args(sr_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                     const sr_box *box, double cell, float r_max, float eps, const float *poly,
                     Geom *g)
{
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n=%lld out of range", (long long)n);
    if (n > 0 && (!x || !y || !z))
        return sr_fail(ctx, SR_EINVAL, "NULL coordinate pointer");
    if (!poly)
        return sr_fail(ctx, SR_EINVAL, "poly is NULL");
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(poly[k]))
            return sr_fail(ctx, SR_EINVAL, "poly[%d] is not finite", k);
    if (!(r_max > 0.f) || !std::isfinite(r_max))
        return sr_fail(ctx, SR_EINVAL, "r_max must be > 0");
    if (!(eps >= 1e-20f) || !std::isfinite(eps))
        return sr_fail(ctx, SR_EINVAL, "eps must be >= 1e-20 (a pair at zero distance must stay finite)");
    int rc = sr_make_geom(ctx, box, cell, g);
    if (rc)
        return rc;
    for (int d = 0; d < 3; ++d) {
        double cs = g->len[d] / g->nc[d];  // chaining cell width
        if ((double)r_max > cs)
            return sr_fail(ctx, SR_EINVAL,
                           "r_max=%g exceeds the cell width %g on axis %d: 27 cells would not cover the cutoff",
                           (double)r_max, cs, d);
        if (g->periodic && g->nc[d] < 3)
            return sr_fail(ctx, SR_EINVAL, "periodic box needs >= 3 cells per axis (axis %d has %d)",
                           d, g->nc[d]);
        if (g->periodic && !(2.0 * (double)r_max < g->len[d]))
            return sr_fail(ctx, SR_EINVAL, "periodic box needs 2 r_max < L");
    }
    // the pair loop's own (x-split) mesh
    return sr_make_geom(ctx, box, cell, g, ctx ? ctx->xsplit : kMaxXsplit);
}

ForceParams make_params(float r_max, float eps, const float *poly)
{
    // p(s) = q(s + eps): q_k = sum_{j >= k} C(j, k) c_j (-eps)^(j - k), in FP64
    static const double C[6][6] = {{1, 0, 0, 0, 0, 0},  {1, 1, 0, 0, 0, 0},
                                   {1, 2, 1, 0, 0, 0},  {1, 3, 3, 1, 0, 0},
                                   {1, 4, 6, 4, 1, 0},  {1, 5, 10, 10, 5, 1}};
    const double e = (double)eps;
    double q[6];
    for (int k = 0; k < 6; ++k) {
        double acc = 0.0;
        for (int j = k; j < 6; ++j)
            acc += C[j][k] * (double)poly[j] * std::pow(-e, j - k);
        q[k] = acc;
    }
    ForceParams fp;
    fp.eps = eps;
    fp.rcut = (float)((double)r_max * (double)r_max + e);
    fp.q0 = (float)q[0];
    fp.nq[0] = 0.f;
    for (int k = 1; k < 6; ++k)
        fp.nq[k] = (float)(-q[k]);
    return fp;
}

// Bin, gather and build work items (everything before the pair loop).
int prepare(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *m, int n,
            const Geom &g, ForceScratch &s)
{
    Bump sz{nullptr, 0, 0};
    force_layout(sz, n, g, s);
    int rc = sr_arena_reserve(ctx, sz.off);
    if (rc)
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    force_layout(b, n, g, s);
    if ((rc = bin_enqueue(ctx, x, y, z, m, n, g, s.bin, s.offsets, s.perm, s.sorted,
                          s.chunk_count)))
        return rc;
    if ((rc = scan_enqueue(ctx, s.chunk_count, g.ncell, s.scan_part2, s.item_off)))
        return rc;
    hipLaunchKernelGGL(k_items, dim3((g.ncell + 255) / 256), dim3(256), 0, ctx->stream, s.offsets,
                       s.item_off, g.ncell, s.items);
    return sr_check_launch(ctx, "k_items");
}

unsigned item_grid(int64_t n, int ncell)
{
    int64_t ub = item_bound(n, ncell);
    return (unsigned)((ub + 7) & ~int64_t(7));
}

}  // namespace

extern "C" int sr_scratch_bytes(const sr_box *box, double cell, int64_t n, int with_force,
                                size_t *bytes)
{
    if (!bytes || n < 0 || n > INT_MAX)
        return SR_EINVAL;
    Geom g;
    // with_force: the largest x split any context may use
    if (sr_make_geom(nullptr, box, cell, &g, with_force ? kMaxXsplit : 1))
        return SR_EINVAL;
    Bump sz{nullptr, 0, 0};
    if (with_force) {
        ForceScratch s;
        force_layout(sz, n, g, s);
    } else {
        BinScratch s;
        bin_layout(sz, n, g, s);
    }
    *bytes = sz.off;
    return SR_OK;
}

extern "C" int sr_force(sr_ctx *ctx, const float *x, const float *y, const float *z,
                        const float *mass, int64_t n, const sr_box *box, double cell, float r_max,
                        float eps, const float poly[6], float *ax, float *ay, float *az,
                        double *momentum3)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    Geom g;
    int rc = check_force_args(ctx, x, y, z, n, box, cell, r_max, eps, poly, &g);
    if (rc)
        return rc;
    if (n > 0 && (!mass || !ax || !ay || !az))
        return sr_fail(ctx, SR_EINVAL, "NULL mass or output pointer");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    ForceScratch s;
    const int rec = sr_timing_begin(ctx);
    sr_timing_mark(ctx, rec, 0);
    if ((rc = prepare(ctx, x, y, z, mass, (int)n, g, s)))
        return rc;
    const ForceParams fp = make_params(r_max, eps, poly);
    sr_timing_mark(ctx, rec, 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_force, dim3(item_grid(n, g.ncell)), dim3(64), 0, ctx->stream,
                           s.items, s.item_off + g.ncell, s.sorted, s.offsets, s.perm,
                           s.bin.mass_mixed, g, fp, ax, ay, az);
        if ((rc = sr_check_launch(ctx, "k_force")))
            return rc;
    }
    sr_timing_mark(ctx, rec, 2);
    if (momentum3) {
        hipLaunchKernelGGL(k_momentum_partial, dim3(kRedBlocks), dim3(256), 0, ctx->stream, mass,
                           ax, ay, az, (int)n, s.mom_part);
        hipLaunchKernelGGL(k_momentum_final, dim3(1), dim3(64), 0, ctx->stream, s.mom_part,
                           momentum3);
        if ((rc = sr_check_launch(ctx, "k_momentum")))
            return rc;
    }
    return SR_OK;
}

extern "C" int sr_pair_stats(sr_ctx *ctx, const float *x, const float *y, const float *z,
                             int64_t n, const sr_box *box, double cell, float r_max,
                             int32_t *per_target, int64_t *useful, int64_t *candidates)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (!useful || !candidates)
        return sr_fail(ctx, SR_EINVAL, "NULL result pointer");
    static const float zero_poly[6] = {0, 0, 0, 0, 0, 0};
    Geom g;
    int rc = check_force_args(ctx, x, y, z, n, box, cell, r_max, 1.0f, zero_poly, &g);
    if (rc)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    // masses are not needed; the gather reads x as a stand-in (w is unused)
    ForceScratch s;
    if ((rc = prepare(ctx, x, y, z, x, (int)n, g, s)))
        return rc;
    // eps = 0 so that se = s and the test is s < r_max^2 exactly as in sr_force
    ForceParams fp = make_params(r_max, 0.0f, zero_poly);
    unsigned long long *st = (unsigned long long *)ctx->stats;
    if ((rc = fill_enqueue(ctx, (int *)st, 0, 4)))
        return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_pair_stats, dim3((unsigned)item_bound(n, g.ncell)), dim3(64), 0,
                           ctx->stream, s.items, s.item_off + g.ncell, s.sorted, s.offsets,
                           s.perm, g, fp, per_target, st);
        if ((rc = sr_check_launch(ctx, "k_pair_stats")))
            return rc;
    }
    unsigned long long h[2] = {0, 0};
    if (hipMemcpyAsync(h, st, sizeof h, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "reading pair statistics failed");
    *useful = (int64_t)h[0];
    *candidates = (int64_t)h[1];
    return SR_OK;
}
