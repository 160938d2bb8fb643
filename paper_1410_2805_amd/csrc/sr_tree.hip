// RCB-tree short-range pass (Sec. 2.4 RCB tree, Sec. 3.1 one tree per fixed
// bin, leaf-node interaction lists shared by the leaf's particles).
//
// After the chaining-mesh binning (the fixed bins of the short-range scale)
// every bin holding more than leaf_max particles is cut into an RCB tree by
// one workgroup: a node's bounding box and FP64 centre of mass are reduced,
// the plane through the centre perpendicular to the longest side splits it,
// and a stable partition of the sorted float4 copy and its permutation keeps
// each child contiguous; the split recurses depth first until a node holds at
// most leaf_max particles.  Leaves are then contiguous ranges of the sorted
// order; a flag at each leaf start, one scan, and per-leaf bounding boxes
// follow.
//
// The force: one wavefront per chunk (<= 64 targets) of a leaf.  Its
// interaction list is every leaf of the 27 neighbouring bins whose bounding
// box (with the bin's periodic image shift) comes within r_max of the target
// leaf's box; accepted leaves are compacted by ballot into the source pieces
// of the chaining-mesh pair loop (up to 64 at a time) and staged through LDS
// exactly as there.  Each sum has a fixed order: deterministic.
#include <climits>
#include <cmath>

#include "sr_internal.h"
#include "sr_pair.h"

namespace {

constexpr int kTB = 256;          // threads of a tree-building block
constexpr int kMaxDepth = 32;     // deeper nodes are leaves
constexpr int kStack = kMaxDepth + 2;

struct TreeScratch {
    float4 *tmp4;       // [n] partition staging
    int *tmpi;          // [n]
    int *flag;          // [n] 1 at the first slot of each leaf
    int *lscan;         // [n + 1] exclusive scan of flag (lscan[n] = leaves)
    int *scan_part;
    int *leaf_start;    // [n + 1] first slot of each leaf; leaf_start[leaves] = n
    int *leaf_cell;     // [n]
    float4 *leaf_lo;    // [n] bounding boxes
    float4 *leaf_hi;    // [n]
    int *cell_leaf;     // [ncell + 1] first leaf of each bin
    int *chunks;        // [n] work items per leaf
    int *item_off;      // [n + 1]
    int *scan_part2;
    int4 *items;        // [n + n / 16 + 1] in leaf order
    int *item_cost;     // [same] cost bucket floor(log2(neighbour-bin sources / S + 64))
    int4 *items_lpt;    // [same] longest first
    int *flag0;         // [1] scan flag (kept 0)
};

int64_t tree_item_bound(int64_t n) { return n + n / 16 + 1; }

void tree_layout(Bump &b, int64_t n, int64_t ncell, TreeScratch &t)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    t.tmp4 = b.take<float4>(nn);
    t.tmpi = b.take<int>(nn);
    t.flag = b.take<int>(nn);
    t.lscan = b.take<int>(nn + 1);
    scan_layout(b, (int)nn, &t.scan_part);
    t.leaf_start = b.take<int>(nn + 1);
    t.leaf_cell = b.take<int>(nn);
    t.leaf_lo = b.take<float4>(nn);
    t.leaf_hi = b.take<float4>(nn);
    t.cell_leaf = b.take<int>((size_t)ncell + 1);
    t.chunks = b.take<int>(nn);
    t.item_off = b.take<int>(nn + 1);
    scan_layout(b, (int)nn, &t.scan_part2);
    t.items = b.take<int4>((size_t)tree_item_bound(n));
    t.item_cost = b.take<int>((size_t)tree_item_bound(n));
    t.items_lpt = b.take<int4>((size_t)tree_item_bound(n));
    t.flag0 = b.take<int>(1);
}

__device__ __forceinline__ float coord(const float4 &p, int axis)
{
    return axis == 0 ? p.x : (axis == 1 ? p.y : p.z);
}

// Block-wide sums and extrema through wave shuffles and one LDS round.
struct Red {
    double d[8];
    float lo[3], hi[3];
    int i;
};

__device__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ float wave_min_f(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan of v over the block (kTB threads); *total = block sum.
__device__ int block_excl(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d)
            inc += t;
    }
    if (lane == 63)
        sh[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int k = 0; k < kTB / 64; ++k) {
        const int s = sh[k];
        base += k < w ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return inc - v + base;
}

// One workgroup per bin: RCB tree of the bin's slots [s0, s0 + n).  Every
// non-empty bin flags its first slot; split nodes flag their leaves' starts.
__global__ __launch_bounds__(kTB) void k_tree_build(int ctot, const int *__restrict__ offsets,
                                                    float4 *__restrict__ sorted,
                                                    int *__restrict__ perm,
                                                    float4 *__restrict__ tmp4,
                                                    int *__restrict__ tmpi,
                                                    int *__restrict__ flag, int leaf_max)
{
    __shared__ int stk_s[kStack], stk_c[kStack], stk_d[kStack];
    __shared__ int sp;
    __shared__ Red part[kTB / 64];
    __shared__ int shs[kTB / 64];
    __shared__ int node[4];   // s, c, depth, split axis (-1: leaf)
    __shared__ double split;
    const int cell = blockIdx.x;
    if (cell >= ctot)
        return;
    const int s0 = offsets[cell], n = offsets[cell + 1] - s0;
    if (n == 0)
        return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) {
        flag[s0] = 1;
        stk_s[0] = s0;
        stk_c[0] = n;
        stk_d[0] = 0;
        sp = n > leaf_max ? 1 : 0;
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) {
            if (sp > 0) {
                --sp;
                node[0] = stk_s[sp];
                node[1] = stk_c[sp];
                node[2] = stk_d[sp];
            } else {
                node[1] = -1;
            }
        }
        __syncthreads();
        const int s = node[0], c = node[1], depth = node[2];
        if (c < 0)
            break;
        if (c <= leaf_max || depth >= kMaxDepth) {
            if (tid == 0)
                flag[s] = 1;
            __syncthreads();
            continue;
        }
        // bounding box and centre of mass (FP64)
        float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
        double mt = 0.0, mx[3] = {0.0, 0.0, 0.0}, gx[3] = {0.0, 0.0, 0.0};
        for (int i = tid; i < c; i += kTB) {
            const float4 p = sorted[s + i];
            const float q[3] = {p.x, p.y, p.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], q[a]);
                hi[a] = fmaxf(hi[a], q[a]);
                mx[a] += (double)p.w * (double)q[a];
                gx[a] += (double)q[a];
            }
            mt += (double)p.w;
        }
        mt = wave_sum_d(mt);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = wave_min_f(lo[a]);
            hi[a] = wave_max_f(hi[a]);
            mx[a] = wave_sum_d(mx[a]);
            gx[a] = wave_sum_d(gx[a]);
        }
        if (lane == 0) {
            part[w].d[0] = mt;
            for (int a = 0; a < 3; ++a) {
                part[w].d[1 + a] = mx[a];
                part[w].d[4 + a] = gx[a];
                part[w].lo[a] = lo[a];
                part[w].hi[a] = hi[a];
            }
        }
        __syncthreads();
        if (tid == 0) {
            double M = 0.0, MX[3] = {0, 0, 0}, GX[3] = {0, 0, 0};
            float L[3] = {3.0e38f, 3.0e38f, 3.0e38f}, H[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
            for (int k = 0; k < kTB / 64; ++k) {
                M += part[k].d[0];
                for (int a = 0; a < 3; ++a) {
                    MX[a] += part[k].d[1 + a];
                    GX[a] += part[k].d[4 + a];
                    L[a] = fminf(L[a], part[k].lo[a]);
                    H[a] = fmaxf(H[a], part[k].hi[a]);
                }
            }
            int ax = 0;
            double best = (double)H[0] - (double)L[0];
            for (int a = 1; a < 3; ++a) {
                const double side = (double)H[a] - (double)L[a];
                if (side > best) {
                    best = side;
                    ax = a;
                }
            }
            node[3] = best > 0.0 ? ax : -1;
            split = M > 0.0 ? MX[ax] / M : GX[ax] / (double)c;
        }
        __syncthreads();
        const int ax = node[3];
        const double com = split;
        if (ax < 0) {  // a point: leaf
            if (tid == 0)
                flag[s] = 1;
            __syncthreads();
            continue;
        }
        // lower child size
        int nl = 0;
        for (int i = tid; i < c; i += kTB)
            nl += (double)coord(sorted[s + i], ax) < com ? 1 : 0;
        nl = wave_sum_i(nl);
        if (lane == 0)
            shs[w] = nl;
        __syncthreads();
        nl = 0;
        for (int k = 0; k < kTB / 64; ++k)
            nl += shs[k];
        __syncthreads();
        if (nl == 0 || nl == c) {  // the plane leaves a side empty: leaf
            if (tid == 0)
                flag[s] = 1;
            __syncthreads();
            continue;
        }
        // stable partition through the staging buffers
        int done_low = 0;
        for (int base = 0; base < c; base += kTB) {
            const int i = base + tid;
            const bool in = i < c;
            float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
            int pi = 0;
            bool low = false;
            if (in) {
                p = sorted[s + i];
                pi = perm[s + i];
                low = (double)coord(p, ax) < com;
            }
            int tot;
            const int ex = block_excl(low ? 1 : 0, shs, &tot);
            if (in) {
                const int dst = low ? s + done_low + ex : s + nl + (base - done_low) + (tid - ex);
                tmp4[dst] = p;
                tmpi[dst] = pi;
            }
            done_low += tot;
        }
        __syncthreads();
        for (int i = tid; i < c; i += kTB) {
            sorted[s + i] = tmp4[s + i];
            perm[s + i] = tmpi[s + i];
        }
        __syncthreads();
        if (tid == 0) {
            // depth first, lower child on top
            stk_s[sp] = s + nl;
            stk_c[sp] = c - nl;
            stk_d[sp] = depth + 1;
            ++sp;
            stk_s[sp] = s;
            stk_c[sp] = nl;
            stk_d[sp] = depth + 1;
            ++sp;
        }
        __syncthreads();
    }
}

// Leaf starts from the flags: leaf_start[l], the leaf's bin, and the end
// marker; the first leaf of each bin.
__global__ __launch_bounds__(256) void k_leaf_compact(int n, int ctot, const int *__restrict__ flag,
                                                      const int *__restrict__ lscan,
                                                      const int *__restrict__ offsets,
                                                      const int *__restrict__ perm,
                                                      const int *__restrict__ cid,
                                                      int *__restrict__ leaf_start,
                                                      int *__restrict__ leaf_cell,
                                                      int *__restrict__ cell_leaf)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && flag[i]) {
        const int l = lscan[i];
        leaf_start[l] = i;
        leaf_cell[l] = cid[perm[i]];
    }
    if (i == 0)
        leaf_start[lscan[n]] = n;
    if (i <= ctot)
        cell_leaf[i] = lscan[offsets[i]];
}

// Per leaf (grid-stride): bounding box by one wavefront, and the number of
// work items (chunks of <= 64 targets).
__global__ __launch_bounds__(64) void k_leaf_boxes(int n, const int *__restrict__ lscan,
                                                   const int *__restrict__ leaf_start,
                                                   const float4 *__restrict__ sorted,
                                                   float4 *__restrict__ leaf_lo,
                                                   float4 *__restrict__ leaf_hi,
                                                   int *__restrict__ chunks)
{
    const int nleaves = lscan[n];
    const int lane = threadIdx.x;
    for (int l = blockIdx.x; l < n; l += gridDim.x) {
        if (l >= nleaves) {
            if (lane == 0)
                chunks[l] = 0;
            continue;
        }
        const int a = leaf_start[l], e = leaf_start[l + 1];
        float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
        for (int k = a + lane; k < e; k += 64) {
            const float4 p = sorted[k];
            lo[0] = fminf(lo[0], p.x);
            lo[1] = fminf(lo[1], p.y);
            lo[2] = fminf(lo[2], p.z);
            hi[0] = fmaxf(hi[0], p.x);
            hi[1] = fmaxf(hi[1], p.y);
            hi[2] = fmaxf(hi[2], p.z);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = wave_min_f(lo[d]);
            hi[d] = wave_max_f(hi[d]);
        }
        if (lane == 0) {
            leaf_lo[l] = make_float4(lo[0], lo[1], lo[2], 0.f);
            leaf_hi[l] = make_float4(hi[0], hi[1], hi[2], 0.f);
            // chunks of at most 64 targets: larger chunks at two targets per
            // lane measured slower here (fewer, longer items)
            chunks[l] = tree_chunks(e - a);
        }
    }
}

// Items {leaf, first slot, targets, S | (tpl - 1) << 5}, shaped by item_shape
// (one or two targets per lane), grid-stride over leaves, each with a cost
// bucket: the sources of the 27 neighbouring bins (an upper bound of the
// interaction list) times the shape's cost per source, plus fixed overhead.
__global__ __launch_bounds__(256) void k_leaf_items(Batch B, int n, const int *__restrict__ lscan,
                                                    const int *__restrict__ leaf_start,
                                                    const int *__restrict__ leaf_cell,
                                                    const int *__restrict__ offsets,
                                                    const int *__restrict__ item_off,
                                                    int4 *__restrict__ items,
                                                    int *__restrict__ item_cost)
{
    const int nleaves = lscan[n];
    const Geom &g = B.one.g;
    for (int l = blockIdx.x * 256 + threadIdx.x; l < nleaves; l += gridDim.x * 256) {
        const int a = leaf_start[l], len = leaf_start[l + 1] - a;
        const int q = item_off[l + 1] - item_off[l];
        int cx, cy, cz;
        decode_cell(leaf_cell[l], g, cx, cy, cz);
        long long src = 0;
        for (int nb = 0; nb < 27; ++nb) {
            int v[3] = {cx + nb % 3 - 1, cy + (nb / 3) % 3 - 1, cz + nb / 9 - 1};
            bool ok = true;
            for (int d = 0; d < 3; ++d) {
                if (g.periodic)
                    v[d] = v[d] < 0 ? v[d] + g.nc[d] : (v[d] >= g.nc[d] ? v[d] - g.nc[d] : v[d]);
                else
                    ok = ok && v[d] >= 0 && v[d] < g.nc[d];
            }
            if (ok) {
                const int id = v[0] + g.nc[0] * (v[1] + g.nc[1] * v[2]);
                src += offsets[id + 1] - offsets[id];
            }
        }
        for (int k = 0; k < q; ++k) {
            const int lo = (int)((long long)k * len / q);
            const int hi = (int)((long long)(k + 1) * len / q);
            int tpl, S;
            const float pass = item_shape(hi - lo, &tpl, &S);
            items[item_off[l] + k] = make_int4(l, a + lo, hi - lo, S | (tpl - 1) << 5);
            const long long cost = (long long)((float)src * pass) + 64;
            item_cost[item_off[l] + k] = 63 - __clzll((unsigned long long)cost);
        }
    }
}

// Leaf of every original particle: the inclusive count of leaf starts - 1.
__global__ __launch_bounds__(256) void k_leaf_of(int n, const int *__restrict__ flag,
                                                 const int *__restrict__ lscan,
                                                 const int *__restrict__ perm,
                                                 int *__restrict__ leaf_of)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        leaf_of[perm[i]] = lscan[i] + flag[i] - 1;
}

// load_tile without the image shifts: entry q = lane + 64 k in pre[k]; entries past
// cnt are far, massless padding.  Returns each entry's piece in byte k, for
// shift_tile.  Nothing here reads the loaded values, so the loads stay in
// flight (behind the previous tile's pair loop) until shift_tile.  This
// holds the loads' registers longer: the tree pass, whose occupancy is set by
// its interaction-list code, gains from it; the mesh pass would lose the
// occupancy step it sits on and keeps load_tile (sr_pair.h).
__device__ __forceinline__ unsigned load_tile_deferred(float4 (&pre)[kTile / 64],
                                                       const Stencil &st,
                                                       const float4 *__restrict__ sorted,
                                                       int g0, int cnt, int lane, int &p)
{
    unsigned pk = 0u;
#pragma unroll
    for (int k = 0; k < kTile / 64; ++k) {
        const int q = lane + 64 * k;
        float4 v = make_float4(kFar, kFar, kFar, 0.f);
        if (q < cnt) {
            const int gi = g0 + q;
            while (gi >= st.pbeg[p + 1])
                ++p;
            v = sorted[st.psrc[p] + (gi - st.pbeg[p])];
            pk |= (unsigned)p << (8 * k);
        }
        pre[k] = v;
    }
    return pk;
}

// Adds the image shift of each entry's piece (kMaxPieces <= 256 fits a byte).
// Padding entries carry piece 0, which exists whenever a tile is loaded; a
// shift of at most one box side (<= 131072) leaves them far outside every
// box.
__device__ __forceinline__ void shift_tile(float4 (&pre)[kTile / 64], unsigned pk,
                                           const Stencil &st)
{
#pragma unroll
    for (int k = 0; k < kTile / 64; ++k) {
        const float4 sh = st.psh[(pk >> (8 * k)) & 255u];
        pre[k].x += sh.x;
        pre[k].y += sh.y;
        pre[k].z += sh.z;
    }
}

// The pair loop of one leaf chunk (one wavefront; single-box batch).
__device__ void process_leaf_item(const Batch &B, const int4 item,
                                  const float4 *__restrict__ sorted, const int *__restrict__ perm,
                                  const int *__restrict__ mass_mixed,
                                  const int *__restrict__ leaf_start,
                                  const int *__restrict__ leaf_cell,
                                  const float4 *__restrict__ leaf_lo,
                                  const float4 *__restrict__ leaf_hi,
                                  const int *__restrict__ cell_leaf, const ForceParams &fp,
                                  float accept2, float4 *tile, Stencil &st, int lane)
{
    const int leaf = item.x, kb = item.y, nt = item.z, S = item_split(item);
    const BoxDesc &d = B.one;
    const Geom &g = d.g;
    int cx, cy, cz;
    decode_cell(leaf_cell[leaf], g, cx, cy, cz);
    const int cc[3] = {cx, cy, cz};
    float F[3];
    frame_shift(g, cc, F);
    const float4 tl = leaf_lo[leaf], th = leaf_hi[leaf];
    const float tlo[3] = {tl.x + F[0], tl.y + F[1], tl.z + F[2]};
    const float thi[3] = {th.x + F[0], th.y + F[1], th.z + F[2]};

    // two targets per lane: lane t of a group holds targets t and t + ln
    const bool two = item_two(item);
    const int ln = two ? (nt + 1) >> 1 : nt;
    const int part = lane_group(lane, ln);
    const int t = lane - part * ln;
    const bool has_target = part < S;
    const bool has2 = two && has_target && t + ln < nt;
    const float4 pt = sorted[kb + t];
    const float4 pt2 = sorted[kb + (has2 ? t + ln : t)];
    const bool pas = is_passive(pt, g);
    const bool pas2 = is_passive(pt2, g);
    const float xi = pt.x + F[0], yi = pt.y + F[1], zi = pt.z + F[2];
    const float xj = pt2.x + F[0], yj = pt2.y + F[1], zj = pt2.z + F[2];
    const bool uniform = mass_mixed[0] == 0;
    const bool work = __any((has_target && !pas) || (has2 && !pas2));
    const int quantum = 4 * S;
    const int cap = kItemTab.cap[S];
    const int qrecip = kItemTab.qrecip[S];
    // the leaf's box holds every target of the chunk (it is the exact float
    // min/max of the leaf's particles, and adding F is monotone): sources
    // beyond the cutoff of all of it are dropped before the pair loop
    TargetBox tb;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        tb.lo[a] = tlo[a];
        tb.hi[a] = thi[a];
    }
    float acx = 0.f, acy = 0.f, acz = 0.f;
    float bcx = 0.f, bcy = 0.f, bcz = 0.f;
    int npiece = 0, total = 0;

    // runs the staged pieces through the pair loop and empties the list
    auto flush = [&]() {
        if (lane == 0)
            st.pbeg[npiece] = total;
        __syncthreads();
        if (work && total > 0) {
            float4 pre[kTile / 64];
            int p = 0, g0 = 0;
            int cnt = total < cap ? total : cap;
            unsigned pk = load_tile_deferred(pre, st, sorted, g0, cnt, lane, p);
            for (;;) {
                shift_tile(pre, pk, st);
                const int nq =
                    quanta_of(store_tile_kept(tile, pre, tb, fp, lane), quantum, qrecip);
                __syncthreads();
                const int g1 = g0 + cnt;
                const int cnt1 = total - g1 < cap ? total - g1 : cap;
                if (cnt1 > 0)
                    pk = load_tile_deferred(pre, st, sorted, g1, cnt1, lane, p);
                const int slice = 4 * nq;
                const float4 *src = tile + (has_target ? part : 0) * slice;
                float tx = 0.f, ty = 0.f, tz = 0.f;
                if (two) {
                    float ux = 0.f, uy = 0.f, uz = 0.f;
                    if (uniform)
                        pair_tile2<true>(src, slice, xi, yi, zi, xj, yj, zj, fp, tx, ty, tz, ux,
                                         uy, uz);
                    else
                        pair_tile2<false>(src, slice, xi, yi, zi, xj, yj, zj, fp, tx, ty, tz, ux,
                                          uy, uz);
                    bcx += ux;
                    bcy += uy;
                    bcz += uz;
                } else if (uniform) {
                    pair_tile<true>(src, slice, xi, yi, zi, fp, tx, ty, tz);
                } else {
                    pair_tile<false>(src, slice, xi, yi, zi, fp, tx, ty, tz);
                }
                acx += tx;
                acy += ty;
                acz += tz;
                __syncthreads();
                if (cnt1 <= 0)
                    break;
                g0 = g1;
                cnt = cnt1;
            }
        }
        __syncthreads();
        npiece = 0;
        total = 0;
    };

    for (int nb = 0; nb < 27; ++nb) {
        const int del[3] = {nb % 3 - 1, (nb / 3) % 3 - 1, nb / 9 - 1};
        int id3[3];
        float sh[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int v = cc[a] + del[a];
            float s = F[a];
            if (g.periodic) {
                if (v < 0) {
                    v += g.nc[a];
                    s -= g.lenf[a];
                } else if (v >= g.nc[a]) {
                    v -= g.nc[a];
                    s += g.lenf[a];
                }
            } else if (v < 0 || v >= g.nc[a]) {
                ok = false;
            }
            id3[a] = v;
            sh[a] = s;
        }
        if (!ok)
            continue;
        const int id = id3[0] + g.nc[0] * (id3[1] + g.nc[1] * id3[2]);
        const int l0 = cell_leaf[id], l1 = cell_leaf[id + 1];
        for (int lb = l0; lb < l1; lb += 64) {
            const int l = lb + lane;
            bool acc = false;
            int len = 0, src = 0;
            if (l < l1) {
                const float4 sl = leaf_lo[l], shh = leaf_hi[l];
                const float slo[3] = {sl.x + sh[0], sl.y + sh[1], sl.z + sh[2]};
                const float shi[3] = {shh.x + sh[0], shh.y + sh[1], shh.z + sh[2]};
                float d2 = 0.f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float gap = fmaxf(0.f, fmaxf(slo[a] - thi[a], tlo[a] - shi[a]));
                    d2 = fmaf(gap, gap, d2);
                }
                acc = d2 < accept2;
                src = leaf_start[l];
                len = leaf_start[l + 1] - src;
            }
            const unsigned long long bal = __ballot(acc);
            const int k = __popcll(bal);
            if (k == 0)
                continue;
            if (npiece + k > kMaxPieces)
                flush();
            int tot;
            const int ex = wave_exclusive_scan(acc ? len : 0, lane, &tot);
            if (acc) {
                const int slot = npiece + __popcll(bal & ((1ull << lane) - 1ull));
                st.psrc[slot] = src;
                st.pbeg[slot] = total + ex;
                st.psh[slot] = make_float4(sh[0], sh[1], sh[2], 0.f);
            }
            npiece += k;
            total += tot;
        }
    }
    flush();
    if (uniform) {
        acx *= pt.w;
        acy *= pt.w;
        acz *= pt.w;
        bcx *= pt2.w;
        bcy *= pt2.w;
        bcz *= pt2.w;
    }
    tile[lane] = make_float4(acx, acy, acz, 0.f);
    tile[64 + lane] = make_float4(bcx, bcy, bcz, 0.f);
    __syncthreads();
    if (part == 0) {
        for (int q = 1; q < S; ++q) {
            const float4 o = tile[t + q * ln];
            acx += o.x;
            acy += o.y;
            acz += o.z;
        }
        const int orig = perm[kb + t];
        d.ax[orig] = pas ? 0.f : acx;
        d.ay[orig] = pas ? 0.f : acy;
        d.az[orig] = pas ? 0.f : acz;
        if (has2) {
            for (int q = 1; q < S; ++q) {
                const float4 o = tile[64 + t + q * ln];
                bcx += o.x;
                bcy += o.y;
                bcz += o.z;
            }
            const int orig2 = perm[kb + t + ln];
            d.ax[orig2] = pas2 ? 0.f : bcx;
            d.ay[orig2] = pas2 ? 0.f : bcy;
            d.az[orig2] = pas2 ? 0.f : bcz;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(64) void k_force_tree(Batch B, const int4 *__restrict__ items,
                                                   const int *__restrict__ n_items,
                                                   const float4 *__restrict__ sorted,
                                                   const int *__restrict__ perm,
                                                   const int *__restrict__ mass_mixed,
                                                   const int *__restrict__ leaf_start,
                                                   const int *__restrict__ leaf_cell,
                                                   const float4 *__restrict__ leaf_lo,
                                                   const float4 *__restrict__ leaf_hi,
                                                   const int *__restrict__ cell_leaf,
                                                   ForceParams fp, float accept2)
{
    __shared__ float4 tile[kTile];
    __shared__ Stencil st;
    const int n = *n_items;
    for (int it = blockIdx.x; it < n; it += gridDim.x)
        process_leaf_item(B, items[it], sorted, perm, mass_mixed, leaf_start, leaf_cell, leaf_lo,
                          leaf_hi, cell_leaf, fp, accept2, tile, st, threadIdx.x);
}

int blocks_of(int64_t count, int per)
{
    const int64_t b = (count + per - 1) / per;
    return (int)(b < 1 ? 1 : b);
}

// Binning, tree build and leaf tables (everything before the pair loop).
int tree_prep(sr_ctx *ctx, const Batch &B, const ForceScratch &s, const TreeScratch &t,
              int leaf_max)
{
    int rc;
    const int n = B.ntot;
    if ((rc = bin_enqueue(ctx, B, s.bin, s.offsets, s.perm, s.sorted, nullptr, nullptr)))
        return rc;
    if ((rc = fill_enqueue(ctx, t.flag, 0, n > 0 ? n : 1)) || (rc = fill_enqueue(ctx, t.flag0, 0, 1)))
        return rc;
    hipLaunchKernelGGL(k_tree_build, dim3(B.ctot > 0 ? B.ctot : 1), dim3(kTB), 0, ctx->stream,
                       B.ctot, s.offsets, s.sorted, s.perm, t.tmp4, t.tmpi, t.flag, leaf_max);
    if ((rc = sr_check_launch(ctx, "k_tree_build")))
        return rc;
    if ((rc = scan_enqueue(ctx, t.flag, n, t.scan_part, t.lscan, t.flag0)))
        return rc;
    const int64_t m = (int64_t)(n > B.ctot ? n : B.ctot) + 1;
    hipLaunchKernelGGL(k_leaf_compact, dim3(blocks_of(m, 256)), dim3(256), 0, ctx->stream, n,
                       B.ctot, t.flag, t.lscan, s.offsets, s.perm, s.bin.cid, t.leaf_start,
                       t.leaf_cell, t.cell_leaf);
    return sr_check_launch(ctx, "k_leaf_compact");
}

int tree_items(sr_ctx *ctx, const Batch &B, const ForceScratch &s, const TreeScratch &t)
{
    int rc;
    const int n = B.ntot;
    const int grid = n < 65536 ? (n > 0 ? n : 1) : 65536;
    hipLaunchKernelGGL(k_leaf_boxes, dim3(grid), dim3(64), 0, ctx->stream, n, t.lscan,
                       t.leaf_start, s.sorted, t.leaf_lo, t.leaf_hi, t.chunks);
    if ((rc = sr_check_launch(ctx, "k_leaf_boxes")))
        return rc;
    if ((rc = scan_enqueue(ctx, t.chunks, n, t.scan_part2, t.item_off, t.flag0)))
        return rc;
    hipLaunchKernelGGL(k_leaf_items, dim3(blocks_of(n, 256) < 4096 ? blocks_of(n, 256) : 4096),
                       dim3(256), 0, ctx->stream, B, n, t.lscan, t.leaf_start, t.leaf_cell,
                       s.offsets, t.item_off, t.items, t.item_cost);
    if ((rc = sr_check_launch(ctx, "k_leaf_items")))
        return rc;
    return lpt_sort_enqueue(ctx, t.items, t.item_cost, t.item_off + n, tree_item_bound(n),
                            s.bin.lpt, t.items_lpt);
}

int tree_setup(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *mass,
               int64_t n, const sr_box *box, double cell, float r_max, int32_t leaf_max,
               float *ax, float *ay, float *az, Batch &B, ForceScratch &s, TreeScratch &t)
{
    if (leaf_max < 1 || leaf_max > (1 << 20))
        return sr_fail(ctx, SR_EINVAL, "leaf_max must be in [1, 2^20]");
    int rc = single_batch(ctx, x, y, z, mass, n, box, cell, r_max, 1, ax, ay, az, &B);
    if (rc)
        return rc;
    if (n > 0 && !mass)
        return sr_fail(ctx, SR_EINVAL, "NULL mass pointer");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    Bump sz{nullptr, 0, 0};
    force_layout(sz, n, B.ctot, 1, s, false, false);  // no work-item sub-items
    tree_layout(sz, n, B.ctot, t);
    if ((rc = sr_arena_reserve(ctx, sz.off)))
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    force_layout(b, n, B.ctot, 1, s, false, false);
    tree_layout(b, n, B.ctot, t);
    return SR_OK;
}

}  // namespace

extern "C" int sr_force_tree(sr_ctx *ctx, const float *x, const float *y, const float *z,
                             const float *mass, int64_t n, const sr_box *box, double cell,
                             float r_max, float eps, const float poly[6], int32_t leaf_max,
                             float *ax, float *ay, float *az, double *momentum3)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    int rc = check_force_params(ctx, r_max, eps, poly);
    if (rc)
        return rc;
    if (n > 0 && (!ax || !ay || !az))
        return sr_fail(ctx, SR_EINVAL, "NULL output pointer");
    Batch B;
    ForceScratch s;
    TreeScratch t;
    if ((rc = tree_setup(ctx, x, y, z, mass, n, box, cell, r_max, leaf_max, ax, ay, az, B, s, t)))
        return rc;
    const int rec = sr_timing_begin(ctx);
    sr_timing_mark(ctx, rec, 0);
    if ((rc = tree_prep(ctx, B, s, t, leaf_max)) || (rc = tree_items(ctx, B, s, t)))
        return rc;
    sr_timing_mark(ctx, rec, 1);
    if (n > 0) {
        const ForceParams fp = make_params(r_max, eps, poly);
        // leaves whose boxes come closer than r_max (with a margin for the
        // float32 box arithmetic) are in the list; the pair cutoff decides
        const float accept2 = (float)((double)r_max * (double)r_max * (1.0 + 1.0 / 4096.0));
        int dev_cus = 256;
        (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
        const int64_t ub = tree_item_bound(n);
        int64_t grid = (int64_t)dev_cus * 32;
        grid = grid < ub ? grid : ub;
        hipLaunchKernelGGL(k_force_tree, dim3((unsigned)grid), dim3(64), 0, ctx->stream, B,
                           t.items_lpt, t.item_off + n, s.sorted, s.perm, s.bin.mass_mixed,
                           t.leaf_start, t.leaf_cell, t.leaf_lo, t.leaf_hi, t.cell_leaf, fp,
                           accept2);
        if ((rc = sr_check_launch(ctx, "k_force_tree")))
            return rc;
    }
    sr_timing_mark(ctx, rec, 2);
    if (momentum3)
        return momentum_enqueue(ctx, B, s.mom_part, momentum3);
    return SR_OK;
}

extern "C" int sr_tree_leaves(sr_ctx *ctx, const float *x, const float *y, const float *z,
                              const float *mass, int64_t n, const sr_box *box, double cell,
                              int32_t leaf_max, int32_t *leaf_of, int64_t *n_leaves)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (!n_leaves || (n > 0 && !leaf_of))
        return sr_fail(ctx, SR_EINVAL, "NULL output pointer");
    Batch B;
    ForceScratch s;
    TreeScratch t;
    // r_max only enters the geometry check: the cell itself
    int rc = tree_setup(ctx, x, y, z, mass, n, box, cell, (float)cell, leaf_max, nullptr, nullptr,
                        nullptr, B, s, t);
    if (rc)
        return rc;
    if ((rc = tree_prep(ctx, B, s, t, leaf_max)))
        return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_leaf_of, dim3(blocks_of(n, 256)), dim3(256), 0, ctx->stream, (int)n,
                           t.flag, t.lscan, s.perm, leaf_of);
        if ((rc = sr_check_launch(ctx, "k_leaf_of")))
            return rc;
    }
    int cnt = 0;
    if (hipMemcpyAsync(&cnt, t.lscan + (n > 0 ? n : 0), sizeof(int), hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "reading the leaf count failed");
    *n_leaves = n > 0 ? cnt : 0;
    return SR_OK;
}
