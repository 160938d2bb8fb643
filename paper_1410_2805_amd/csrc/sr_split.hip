// Split (cell + float32 offset) coordinates: conversion from and to float64
// positions, and the stream / kick maps of the stream-kick-stream step
// (Sec. 2.5) applied to resident split state.
//
// A coordinate of a periodic box of side L meshed into n_c chaining cells of
// width h = L / n_c is held as c = floor(x / h) (packed 10 bits per axis into
// cell3) and o = fl32(x - c h) in [0, h).  Offsets carry ulp(h) rounding
// instead of ulp(L), and the pair loop differences them without forming
// global coordinates (sr_force.hip).
#include <climits>
#include <cmath>

#include "sr_internal.h"
#include "sr_split.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int pack3(const int c[3])
{
    return c[0] | (c[1] << 10) | (c[2] << 20);
}

__device__ __forceinline__ void unpack3(int p, int c[3])
{
    c[0] = p & 1023;
    c[1] = (p >> 10) & 1023;
    c[2] = (p >> 20) & 1023;
}

// Re-home an offset that left [0, h): at most a few cells per call (the
// caller keeps |v dt| well below h); wraps the cell index periodically.
__device__ __forceinline__ void rehome(double &o, int &c, double h, int nc)
{
    while (o >= h) {
        o -= h;
        c = c + 1 == nc ? 0 : c + 1;
    }
    while (o < 0.0) {
        o += h;
        c = c == 0 ? nc - 1 : c - 1;
    }
}

__global__ __launch_bounds__(kBlock) void k_from_f64(const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ z, int n,
                                                     SplitGeom sg, int *__restrict__ cell3,
                                                     float *__restrict__ ox,
                                                     float *__restrict__ oy,
                                                     float *__restrict__ oz,
                                                     int *__restrict__ status)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double p[3] = {x[i], y[i], z[i]};
    int c[3];
    float o[3];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (!(p[k] >= 0.0 && p[k] < sg.len[k])) {
            bad = true;
            c[k] = 0;
            o[k] = 0.f;
            continue;
        }
        int ci = (int)floor(p[k] * sg.inv[k]);
        ci = ci < sg.nc[k] - 1 ? ci : sg.nc[k] - 1;
        double off = p[k] - (double)ci * sg.h[k];
        rehome(off, ci, sg.h[k], sg.nc[k]);
        c[k] = ci;
        o[k] = (float)off;
    }
    if (bad)
        atomicOr(status, 1);
    cell3[i] = pack3(c);
    ox[i] = o[0];
    oy[i] = o[1];
    oz[i] = o[2];
}

__global__ __launch_bounds__(kBlock) void k_to_f64(const int *__restrict__ cell3,
                                                   const float *__restrict__ ox,
                                                   const float *__restrict__ oy,
                                                   const float *__restrict__ oz, int n,
                                                   SplitGeom sg, double *__restrict__ x,
                                                   double *__restrict__ y,
                                                   double *__restrict__ z)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    int c[3];
    unpack3(cell3[i], c);
    const float o[3] = {ox[i], oy[i], oz[i]};
    double *out[3] = {x, y, z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double v = (double)c[k] * sg.h[k] + (double)o[k];
        if (v >= sg.len[k])
            v -= sg.len[k];
        out[k][i] = v;
    }
}

// Serving state update over all slots of a tick (slot s owns particles
// [start[s], start[s+1]) of the concatenated numbering).
//   mode 0: stream  o += v dt/2 (re-home);
//   mode 1: kick v += a dt, then stream o += v dt/2 (re-home).
__global__ __launch_bounds__(kBlock) void k_slot_update(const SlotState *__restrict__ slots,
                                                        const int *__restrict__ start, int nslot,
                                                        int ntot, int mode)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= ntot)
        return;
    int lo = 0, hi = nslot - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const SlotState &S = slots[lo];
    const int li = i - start[lo];
    float v[3] = {S.vx[li], S.vy[li], S.vz[li]};
    if (mode == 1) {
        v[0] = fmaf(S.ax[li], S.dt, v[0]);
        v[1] = fmaf(S.ay[li], S.dt, v[1]);
        v[2] = fmaf(S.az[li], S.dt, v[2]);
        S.vx[li] = v[0];
        S.vy[li] = v[1];
        S.vz[li] = v[2];
    }
    int c[3];
    unpack3(S.cell3[li], c);
    float *o[3] = {S.ox, S.oy, S.oz};
    const double half = 0.5 * (double)S.dt;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double off = (double)o[k][li] + (double)v[k] * half;
        rehome(off, c[k], S.g.h[k], S.g.nc[k]);
        o[k][li] = (float)off;
    }
    S.cell3[li] = pack3(c);
}

// One box of split state: kick v += a * kick (when a is given), then
// nstream times stream o += v * stream in FP64 with re-homing (stream == 0:
// kick only).  Each stream rounds the offset to float32 as a separate launch
// would, so two streams here are bitwise two launches.  The arithmetic of
// each map is that of k_slot_update.
__global__ __launch_bounds__(kBlock) void k_kick_stream(SplitGeom sg, int n, int *__restrict__ cell3,
                                                        float *__restrict__ ox,
                                                        float *__restrict__ oy,
                                                        float *__restrict__ oz,
                                                        float *__restrict__ vx,
                                                        float *__restrict__ vy,
                                                        float *__restrict__ vz,
                                                        const float *__restrict__ ax,
                                                        const float *__restrict__ ay,
                                                        const float *__restrict__ az, float kick,
                                                        double stream, int nstream)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    float v[3] = {vx[i], vy[i], vz[i]};
    if (ax) {
        v[0] = fmaf(ax[i], kick, v[0]);
        v[1] = fmaf(ay[i], kick, v[1]);
        v[2] = fmaf(az[i], kick, v[2]);
        vx[i] = v[0];
        vy[i] = v[1];
        vz[i] = v[2];
    }
    if (stream == 0.0)
        return;
    int c[3];
    unpack3(cell3[i], c);
    float *o[3] = {ox, oy, oz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float of = o[k][i];
        for (int s = 0; s < nstream; ++s) {
            double off = (double)of + (double)v[k] * stream;
            rehome(off, c[k], sg.h[k], sg.nc[k]);
            of = (float)off;
        }
        o[k][i] = of;
    }
    cell3[i] = pack3(c);
}

// ---- multilevel stepping (Sec. 3.1, Eq. (kicks)) --------------------------

__device__ __forceinline__ int split_cell_index(int packed, const SplitGeom &sg)
{
    int c[3];
    unpack3(packed, c);
    return c[0] + sg.nc[0] * (c[1] + sg.nc[1] * c[2]);
}

// Particles per chaining cell (counts cleared by the caller): a block counts
// its kMlCountPer x kBlock particles per cell in an LDS hash table, then adds
// each distinct cell's count with one global atomic.
constexpr int kMlCountPer = 4;
__global__ __launch_bounds__(kBlock) void k_ml_count(const int *__restrict__ cell3, int n,
                                                     SplitGeom sg, int *__restrict__ counts)
{
    __shared__ int hkey[kHash];
    __shared__ int hcnt[kHash];
    for (int h = threadIdx.x; h < kHash; h += kBlock) {
        hkey[h] = -1;
        hcnt[h] = 0;
    }
    __syncthreads();
    const int base = blockIdx.x * kBlock * kMlCountPer;
#pragma unroll
    for (int k = 0; k < kMlCountPer; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        if (i < n)
            atomicAdd(&hcnt[lds_hash_slot(hkey, split_cell_index(cell3[i], sg))], 1);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kHash; h += kBlock)
        if (hcnt[h] > 0)
            atomicAdd(counts + hkey[h], hcnt[h]);
}

// Kicks per subcycle: l = floor(rho / rho_0) / d + 1 clamped to [lmin, lmax],
// rho / rho_0 = count * ncell / n (FP64).
__global__ __launch_bounds__(kBlock) void k_ml_level(const int *__restrict__ cell3, int n,
                                                     SplitGeom sg, const int *__restrict__ counts,
                                                     int d, int lmin, int lmax,
                                                     unsigned char *__restrict__ level)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const double ncell = (double)sg.nc[0] * sg.nc[1] * sg.nc[2];
    const long long r = (long long)floor((double)counts[split_cell_index(cell3[i], sg)] * ncell /
                                         (double)n);
    long long l = r / d + 1;
    l = l < lmin ? lmin : (l > lmax ? lmax : l);
    level[i] = (unsigned char)l;
}

__device__ __forceinline__ bool ml_kicks(int l, int m, int M)
{
    const int t = 2 * m * l;
    return t % M == 0 && ((t / M) & 1);
}

// Particles that kick after piece m: 1, or 2 above the lowest level.  The
// short-range pass cuts the cells holding a 2 into finer work items: such a
// pass runs over few, dense cells, and one wavefront per large chunk would
// leave most of the GPU idle.
__global__ __launch_bounds__(kBlock) void k_ml_active(const unsigned char *__restrict__ level,
                                                      int n, int m, int M, int lmin,
                                                      unsigned char *__restrict__ active)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        active[i] = ml_kicks(level[i], m, M) ? (level[i] > lmin ? 2 : 1) : 0;
}

// After stream piece m: particles of a level that kicks at m take v += a tau/l
// (when a is given); then every particle streams o += v * stream.
__global__ __launch_bounds__(kBlock) void k_ml_update(SplitGeom sg, int n, int *__restrict__ cell3,
                                                      float *__restrict__ ox,
                                                      float *__restrict__ oy,
                                                      float *__restrict__ oz,
                                                      float *__restrict__ vx,
                                                      float *__restrict__ vy,
                                                      float *__restrict__ vz,
                                                      const float *__restrict__ ax,
                                                      const float *__restrict__ ay,
                                                      const float *__restrict__ az,
                                                      const unsigned char *__restrict__ level,
                                                      int m, int M, double tau, double stream,
                                                      int nstream)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    float v[3] = {vx[i], vy[i], vz[i]};
    const int l = level[i];
    if (ax && ml_kicks(l, m, M)) {
        const float kick = (float)(tau / (double)l);
        v[0] = fmaf(ax[i], kick, v[0]);
        v[1] = fmaf(ay[i], kick, v[1]);
        v[2] = fmaf(az[i], kick, v[2]);
        vx[i] = v[0];
        vy[i] = v[1];
        vz[i] = v[2];
    }
    if (stream == 0.0)
        return;
    int c[3];
    unpack3(cell3[i], c);
    float *o[3] = {ox, oy, oz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float of = o[k][i];
        for (int s = 0; s < nstream; ++s) {
            double off = (double)of + (double)v[k] * stream;
            rehome(off, c[k], sg.h[k], sg.nc[k]);
            of = (float)off;
        }
        o[k][i] = of;
    }
    cell3[i] = pack3(c);
}

// ---- FP64 kinetic energy K = sum_i m_i |v_i|^2 / 2 ---------------------------
// Fixed partition into R contiguous chunks (R = clamp(ceil(n / 4096), 1,
// kRedBlocks)), a fixed tree inside each block and over the partials:
// bitwise reproducible.

__global__ __launch_bounds__(256) void k_kinetic_partial(const float *__restrict__ vx,
                                                         const float *__restrict__ vy,
                                                         const float *__restrict__ vz,
                                                         const float *__restrict__ m, int n,
                                                         double *__restrict__ part)
{
    __shared__ double sh[256];
    int R = (n + 4095) / 4096;
    R = R < 1 ? 1 : (R > kRedBlocks ? kRedBlocks : R);
    const int chunk = (n + R - 1) / R;
    const int lo = blockIdx.x * chunk;
    const int hi = (int)blockIdx.x < R ? (lo + chunk < n ? lo + chunk : n) : lo;
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += 256) {
        const double a = vx[i], b = vy[i], c = vz[i];
        s += 0.5 * (double)m[i] * (a * a + b * b + c * c);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_kinetic_final(const double *__restrict__ part,
                                                       double *__restrict__ out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < kRedBlocks; k += 256)
        s += part[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = sh[0];
}

}  // namespace

int split_geom(sr_ctx *ctx, const sr_box *box, double cell, SplitGeom *sg)
{
    Geom g;
    int rc = sr_make_geom(ctx, box, cell, &g);
    if (rc)
        return rc;
    if (!box->periodic)
        return sr_fail(ctx, SR_EINVAL, "split coordinates need a periodic box");
    for (int d = 0; d < 3; ++d) {
        if (g.nc[d] > kSplitMaxCells)
            return sr_fail(ctx, SR_EINVAL, "split coordinates allow at most %d cells per axis",
                           kSplitMaxCells);
        sg->len[d] = g.len[d];
        sg->inv[d] = g.inv[d];
        sg->h[d] = g.w[d];
        sg->nc[d] = g.nc[d];
    }
    return SR_OK;
}

int split_from_f64_enqueue(sr_ctx *ctx, const double *x, const double *y, const double *z, int n,
                           const SplitGeom &sg, int *cell3, float *ox, float *oy, float *oz)
{
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_from_f64, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       x, y, z, n, sg, cell3, ox, oy, oz, ctx->status);
    return sr_check_launch(ctx, "k_from_f64");
}

int split_to_f64_enqueue(sr_ctx *ctx, const int *cell3, const float *ox, const float *oy,
                         const float *oz, int n, const SplitGeom &sg, double *x, double *y,
                         double *z)
{
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_to_f64, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       cell3, ox, oy, oz, n, sg, x, y, z);
    return sr_check_launch(ctx, "k_to_f64");
}

int slot_update_enqueue(sr_ctx *ctx, const SlotState *slots, const int *start, int nslot,
                        int ntot, int mode)
{
    if (ntot <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_slot_update, dim3((ntot + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       ctx->stream, slots, start, nslot, ntot, mode);
    return sr_check_launch(ctx, "k_slot_update");
}

extern "C" int sr_split_from_f64(sr_ctx *ctx, const double *x, const double *y, const double *z,
                                 int64_t n, const sr_box *box, double cell, int32_t *cell3,
                                 float *ox, float *oy, float *oz)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > INT_MAX || (n > 0 && (!x || !y || !z || !cell3 || !ox || !oy || !oz)))
        return sr_fail(ctx, SR_EINVAL, "bad size or NULL pointer");
    SplitGeom sg;
    int rc = split_geom(ctx, box, cell, &sg);
    if (rc)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    return split_from_f64_enqueue(ctx, x, y, z, (int)n, sg, cell3, ox, oy, oz);
}

extern "C" int sr_split_to_f64(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                               const float *oz, int64_t n, const sr_box *box, double cell,
                               double *x, double *y, double *z)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > INT_MAX || (n > 0 && (!x || !y || !z || !cell3 || !ox || !oy || !oz)))
        return sr_fail(ctx, SR_EINVAL, "bad size or NULL pointer");
    SplitGeom sg;
    int rc = split_geom(ctx, box, cell, &sg);
    if (rc)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    return split_to_f64_enqueue(ctx, cell3, ox, oy, oz, (int)n, sg, x, y, z);
}

int kick_stream_enqueue(sr_ctx *ctx, const SplitGeom &sg, int n, int *cell3, float *ox, float *oy,
                        float *oz, float *vx, float *vy, float *vz, const float *ax,
                        const float *ay, const float *az, float kick, double stream, int nstream)
{
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_kick_stream, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       ctx->stream, sg, n, cell3, ox, oy, oz, vx, vy, vz, ax, ay, az, kick,
                       stream, nstream);
    return sr_check_launch(ctx, "k_kick_stream");
}

int ml_levels_enqueue(sr_ctx *ctx, const SplitGeom &sg, const int *cell3, int n, int *counts,
                      int d, int lmin, int lmax, unsigned char *level)
{
    if (n <= 0)
        return SR_OK;
    const int64_t ncell = (int64_t)sg.nc[0] * sg.nc[1] * sg.nc[2];
    int rc = fill_enqueue(ctx, counts, 0, ncell);
    if (rc)
        return rc;
    const dim3 grid((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_ml_count, dim3((n + kBlock * kMlCountPer - 1) / (kBlock * kMlCountPer)),
                       dim3(kBlock), 0, ctx->stream, cell3, n, sg, counts);
    hipLaunchKernelGGL(k_ml_level, grid, dim3(kBlock), 0, ctx->stream, cell3, n, sg, counts, d,
                       lmin, lmax, level);
    return sr_check_launch(ctx, "k_ml_level");
}

int ml_active_enqueue(sr_ctx *ctx, const unsigned char *level, int n, int m, int M, int lmin,
                      unsigned char *active)
{
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_ml_active, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       level, n, m, M, lmin, active);
    return sr_check_launch(ctx, "k_ml_active");
}

int ml_update_enqueue(sr_ctx *ctx, const SplitGeom &sg, int n, int *cell3, float *ox, float *oy,
                      float *oz, float *vx, float *vy, float *vz, const float *ax,
                      const float *ay, const float *az, const unsigned char *level, int m, int M,
                      double tau, double stream, int nstream)
{
    if (n <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_ml_update, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, ctx->stream,
                       sg, n, cell3, ox, oy, oz, vx, vy, vz, ax, ay, az, level, m, M, tau,
                       stream, nstream);
    return sr_check_launch(ctx, "k_ml_update");
}

int kinetic_enqueue(sr_ctx *ctx, const float *vx, const float *vy, const float *vz,
                    const float *m, int n, double *part, double *out)
{
    hipLaunchKernelGGL(k_kinetic_partial, dim3(kRedBlocks), dim3(256), 0, ctx->stream, vx, vy, vz,
                       m, n, part);
    hipLaunchKernelGGL(k_kinetic_final, dim3(1), dim3(256), 0, ctx->stream, part, out);
    return sr_check_launch(ctx, "k_kinetic");
}

extern "C" int sr_kinetic(sr_ctx *ctx, const float *vx, const float *vy, const float *vz,
                          const float *mass, int64_t n, double *out)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (!out || n < 0 || n > INT_MAX || (n > 0 && (!vx || !vy || !vz || !mass)))
        return sr_fail(ctx, SR_EINVAL, "bad size or NULL pointer");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    int rc = sr_arena_reserve(ctx, kRedBlocks * sizeof(double));
    if (rc)
        return rc;
    return kinetic_enqueue(ctx, vx, vy, vz, mass, (int)n, reinterpret_cast<double *>(ctx->arena),
                           out);
}
