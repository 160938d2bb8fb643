// Pair-loop building blocks shared by the chaining-mesh pass (sr_force.hip)
// and the RCB-tree pass (sr_tree.hip): source pieces, their LDS staging and
// the float32 pair arithmetic of Eq. (force).
#pragma once

#include "sr_internal.h"

namespace {

constexpr int kTile = 256;       // sources per LDS tile (4 KiB)
constexpr float kFar = 1.0e6f;   // padding source far outside any box, mass 0

// Source pieces of one target cell: at most 18 (9 rows, each split where it
// wraps) in global coordinates, at most 63 (one per cell) in split
// coordinates.  pbeg[npiece] = all sources; unused pieces are empty.
constexpr int kMaxPieces = 64;
struct Stencil {
    int pbeg[kMaxPieces + 1];  // prefix of piece lengths
    int psrc[kMaxPieces];      // first sorted slot of each piece
    float4 psh[kMaxPieces];    // shift added to the piece's coordinates
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
// call).  Global coordinates: lanes < 18 each own one piece slot, row r =
// lane/2, half = lane%2, the shift is the periodic image shift.  Split
// coordinates: lanes < 9 (2 hx + 1) each own one cell of the stencil and the
// shift is the cell's offset from the target cell, (dx w0, dy w1, dz w2), so
// coordinates stay cell-relative and periodic wrap needs no shift at all.
__device__ void build_stencil(Stencil &st, const int *__restrict__ offsets, const Geom &g, int cx,
                              int cy, int cz, const float F[3], int lane)
{
    int len = 0, src = 0;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    const int W = 2 * g.hx + 1;
    if (g.split && lane < 9 * W) {
        const int r = lane / W, k = lane - r * W;
        const int dx = k - g.hx, dy = r % 3 - 1, dz = r / 3 - 1;
        int nx = cx + dx, ny = cy + dy, nz = cz + dz;
        nx = nx < 0 ? nx + g.nc[0] : (nx >= g.nc[0] ? nx - g.nc[0] : nx);
        ny = ny < 0 ? ny + g.nc[1] : (ny >= g.nc[1] ? ny - g.nc[1] : ny);
        nz = nz < 0 ? nz + g.nc[2] : (nz >= g.nc[2] ? nz - g.nc[2] : nz);
        const int id = nx + g.nc[0] * (ny + g.nc[1] * nz);
        src = offsets[id];
        len = offsets[id + 1] - src;
        sx = (float)((double)dx * g.w[0]);
        sy = (float)((double)dy * g.w[1]);
        sz = (float)((double)dz * g.w[2]);
    } else if (!g.split && lane < 18) {
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
    st.pbeg[lane] = beg;
    st.psrc[lane] = src;
    st.psh[lane] = make_float4(sx, sy, sz, 0.f);
    if (lane == 0)
        st.pbeg[kMaxPieces] = total;
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
        F[d] = (g.periodic && !g.split && cc[d] + h[d] >= g.nc[d]) ? -g.lenf[d] : 0.f;
}

__device__ __forceinline__ void decode_cell(int cell, const Geom &g, int &cx, int &cy, int &cz)
{
    const int plane = g.nc[0] * g.nc[1];
    cz = div_by(cell, g.div_m[0], g.div_s[0]);
    const int rem = cell - cz * plane;
    cy = div_by(rem, g.div_m[1], g.div_s[1]);
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

// Loads sources [g0, g0 + cnt) of the stencil (cnt <= kTile) into registers,
// entry q = lane + 64 k in pre[k]; entries past cnt are far, massless padding.
__device__ __forceinline__ void load_tile(float4 (&pre)[kTile / 64], const Stencil &st,
                                          const float4 *__restrict__ sorted, int g0, int cnt,
                                          int lane, int &p)
{
#pragma unroll
    for (int k = 0; k < kTile / 64; ++k) {
        const int q = lane + 64 * k;
        float4 v = make_float4(kFar, kFar, kFar, 0.f);
        if (q < cnt) {
            const int gi = g0 + q;
            while (gi >= st.pbeg[p + 1])
                ++p;
            const float4 s = sorted[st.psrc[p] + (gi - st.pbeg[p])];
            const float4 sh = st.psh[p];
            v = make_float4(s.x + sh.x, s.y + sh.y, s.z + sh.z, s.w);
        }
        pre[k] = v;
    }
}

// Bounding box of a work item's targets, for a test that drops stencil
// sources before the pair loop.  The paper's chaining mesh (Sec. 3.1) offers
// every target all particles of its neighbour cells and lets the cutoff
// reject the far ones; the test rejects, per item, sources that are beyond
// the cutoff of the whole box, which changes no sum (see source_kept).
struct TargetBox {
    float lo[3], hi[3];
};

// Order-preserving map between finite float bit patterns and int32 (its own
// inverse): non-negative values keep their bits, negative ones have the
// magnitude bits flipped, so integer order is float order (-0 below +0).
__device__ __forceinline__ int ordered_key(int b)
{
    return b ^ ((b >> 31) & 0x7fffffff);
}

// One step of a row reduction: v combined with lane (ctrl) of its row.
template <int kCtrl, bool kMax>
__device__ __forceinline__ int row_step(int v)
{
    const int o = __builtin_amdgcn_mov_dpp(v, kCtrl, 0xF, 0xF, true);
    return kMax ? max(v, o) : min(v, o);
}

// Minimum (kMax false) or maximum of a and b over the 64 lanes, uniform: on
// ordered keys, within each row of 16 lanes by exchanges across pairs,
// quads, half rows and the row (DPP quad_perm [1,0,3,2], [2,3,0,1], row half
// mirror, row mirror), then across the four rows' first lanes.
template <bool kMax>
__device__ __forceinline__ float wave_extreme(float a, float b)
{
    const int ka = ordered_key(__float_as_int(a)), kb = ordered_key(__float_as_int(b));
    int v = kMax ? max(ka, kb) : min(ka, kb);
    v = row_step<0xB1, kMax>(v);
    v = row_step<0x4E, kMax>(v);
    v = row_step<0x141, kMax>(v);
    v = row_step<0x140, kMax>(v);
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    const int m = kMax ? max(max(r0, r1), max(r2, r3)) : min(min(r0, r1), min(r2, r3));
    // held in a scalar register through the whole item
    return __int_as_float(ordered_key(__builtin_amdgcn_readfirstlane(m)));
}

// Every lane passes the two targets it holds (equal when it holds one); the
// box comes back the same in all lanes.  All 64 lanes must be active.
__device__ __forceinline__ TargetBox target_box(float xi, float yi, float zi, float xj, float yj,
                                                float zj)
{
    TargetBox b;
    b.lo[0] = wave_extreme<false>(xi, xj);
    b.lo[1] = wave_extreme<false>(yi, yj);
    b.lo[2] = wave_extreme<false>(zi, zj);
    b.hi[0] = wave_extreme<true>(xi, xj);
    b.hi[1] = wave_extreme<true>(yi, yj);
    b.hi[2] = wave_extreme<true>(zi, zj);
    return b;
}

// Whether source s can interact with any target in the box: its per-axis gap
// g to the box is at most its distance along that axis to every target in
// it (rounding is monotone), so g^2 summed by the pair loop's own FMA chain,
// with eps, is at most every pair's se.  A source that fails se < rcut here
// fails it for every target of the box: dropping it changes no result.
__device__ __forceinline__ bool source_kept(const float4 &s, const TargetBox &b,
                                            const ForceParams &fp)
{
    const float gx = fmaxf(0.f, fmaxf(b.lo[0] - s.x, s.x - b.hi[0]));
    const float gy = fmaxf(0.f, fmaxf(b.lo[1] - s.y, s.y - b.hi[1]));
    const float gz = fmaxf(0.f, fmaxf(b.lo[2] - s.z, s.z - b.hi[2]));
    return fmaf(gx, gx, fmaf(gy, gy, fmaf(gz, gz, fp.eps))) < fp.rcut;
}

// Per lane-group count S (1..16) of an item: the tile capacity cap[S] (a
// multiple of the slice quantum 4 S) and the quantum's 16-bit fixed-point
// reciprocal qrecip[S], rounded up, for quanta_of; per target count ln
// (1..64) of a group, lnrecip[ln] = ceil(2^16 / ln), for lane_group.  Read
// with a uniform index, so from scalar memory instead of dividing.
struct ItemTables {
    int cap[kMaxSplit + 1];
    int qrecip[kMaxSplit + 1];
    int lnrecip[65];
};

constexpr ItemTables make_item_tables()
{
    ItemTables t{};
    for (int s = 1; s <= kMaxSplit; ++s) {
        const int q = 4 * s;
        t.cap[s] = kTile / q * q;
        t.qrecip[s] = (65536 + q - 1) / q;
    }
    for (int l = 1; l <= 64; ++l)
        t.lnrecip[l] = (65536 + l - 1) / l;
    return t;
}

__constant__ const ItemTables kItemTab = make_item_tables();

// lane / ln for lane < 64 and 1 <= ln <= 64: lane r / 2^16 exceeds lane / ln
// by less than 64 / 2^16 < 1 / 64 <= 1 / ln, which cannot reach the next
// integer.
__device__ __forceinline__ int lane_group(int lane, int ln)
{
    return (lane * kItemTab.lnrecip[ln]) >> 16;
}

// ceil(n / q) for 0 <= n <= kTile from r = ceil(2^16 / q) (qrecip): with x = n + q - 1
// < 320, x r / 2^16 exceeds x / q by less than 320 / 2^16 < 1 / 64 <= 1 / q,
// which cannot reach the next integer.
__device__ __forceinline__ int quanta_of(int n, int q, int r)
{
    return ((n + q - 1) * r) >> 16;
}

// Writes the kTile entries of a tile loaded by load_tile as a stable
// partition: first those that pass source_kept against the box, in load
// order (entry q = lane + 64 k), then all others.  Returns the count of
// kept entries.  An entry that fails the box test fails the pair loop's
// cutoff for every target in the box and adds exactly zero to it (as does
// load_tile's far padding, which always fails), so any prefix of the tile
// that covers the kept entries gives every target the same sum.
__device__ __forceinline__ int store_tile_kept(float4 *tile, const float4 (&pre)[kTile / 64],
                                               const TargetBox &box, const ForceParams &fp,
                                               int lane)
{
    bool kk[kTile / 64];
    unsigned long long bal[kTile / 64];
    int base[kTile / 64];
    int n = 0;
#pragma unroll
    for (int k = 0; k < kTile / 64; ++k) {
        kk[k] = source_kept(pre[k], box, fp);
        bal[k] = __ballot(kk[k]);
        base[k] = n;
        n += __popcll(bal[k]);
    }
#pragma unroll
    for (int k = 0; k < kTile / 64; ++k) {
        // kept entries before this one in load order
        const int kp = base[k] + (int)__builtin_amdgcn_mbcnt_hi(
                                     (unsigned)(bal[k] >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)bal[k], 0u));
        const int q = lane + 64 * k;
        tile[kk[k] ? kp : n + (q - kp)] = pre[k];
    }
    return n;
}

// One pair of Eq. (force) for one lane: source s, target (xi, yi, zi);
// adds f d (times the source mass unless uniform) to tx, ty, tz.
template <bool kUniformMass>
__device__ __forceinline__ void pair_one(const float4 s, float xi, float yi, float zi,
                                         const ForceParams &fp, float &tx, float &ty, float &tz)
{
    const float dx = s.x - xi;
    const float dy = s.y - yi;
    const float dz = s.z - zi;
    // se = s + eps; f = se^(-3/2) - q(se) with q(se) = p(se - eps)
    const float se = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, fp.eps)));
    const float rs = __builtin_amdgcn_rsqf(se);
    const float rs2 = rs * rs;
    const float tt = fmaf(rs2, rs, -fp.q0);
    float h = fmaf(fp.nq[5], se, fp.nq[4]);
    h = fmaf(h, se, fp.nq[3]);
    h = fmaf(h, se, fp.nq[2]);
    h = fmaf(h, se, fp.nq[1]);
    float f = fmaf(h, se, tt);
    f = se < fp.rcut ? f : 0.f;  // cutoff by select: also zeroes padding
    if (!kUniformMass)
        f *= s.w;
    tx = fmaf(f, dx, tx);
    ty = fmaf(f, dy, ty);
    tz = fmaf(f, dz, tz);
}

// One tile of pair interactions for one lane: sources src[0 .. cnt) (cnt a
// multiple of 4), target (xi, yi, zi); partial sums into tx, ty, tz.
template <bool kUniformMass>
__device__ __forceinline__ void pair_tile(const float4 *src, int cnt, float xi, float yi, float zi,
                                          const ForceParams &fp, float &tx, float &ty, float &tz)
{
    for (int j = 0; j < cnt; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            pair_one<kUniformMass>(src[j + u], xi, yi, zi, fp, tx, ty, tz);
    }
}

// pair_tile for two targets per lane: every source read from LDS serves both
// (xi, yi, zi) -> t and (xj, yj, zj) -> u, each summed in source order (cnt
// even; two sources per iteration keep the register count of pair_tile).
template <bool kUniformMass>
__device__ __forceinline__ void pair_tile2(const float4 *src, int cnt, float xi, float yi,
                                           float zi, float xj, float yj, float zj,
                                           const ForceParams &fp, float &tx, float &ty, float &tz,
                                           float &ux, float &uy, float &uz)
{
    for (int j = 0; j < cnt; j += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const float4 s = src[j + u];
            pair_one<kUniformMass>(s, xi, yi, zi, fp, tx, ty, tz);
            pair_one<kUniformMass>(s, xj, yj, zj, fp, ux, uy, uz);
        }
    }
}

// Item layout (item_word): {cell (global), first sorted slot, targets, S |
// two << 5 | sk << 6 | (ns - 1) << 10 | box << 14}, two = 1 when each lane
// holds two targets, sk of ns the sub-item's part of the stencil sources.
__device__ __forceinline__ int item_split(const int4 &it) { return it.w & 31; }
__device__ __forceinline__ bool item_two(const int4 &it) { return (it.w >> 5) & 1; }
__device__ __forceinline__ int item_sub(const int4 &it) { return (it.w >> 6) & 15; }
__device__ __forceinline__ int item_nsub(const int4 &it) { return ((it.w >> 10) & 15) + 1; }
__device__ __forceinline__ int item_box(const int4 &it) { return it.w >> 14; }

}  // namespace
