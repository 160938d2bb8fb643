// Short-range particle-particle force on gfx950 (Eq. (force), Sec. 3.1).
//
// After binning (sr_bin.hip) the particles sit cell by cell in a float4
// (x, y, z, m) copy.  Each force work item is one cell's chunk of at most 128
// targets, or a sub-item taking a consecutive part of that chunk's stencil
// sources.  One wavefront owns an item:
//   - the 27 neighbour cells are 9 rows of 3 cells that are contiguous in the
//     sorted order, so the source list is at most 18 contiguous pieces (a row
//     splits in two where it wraps around a periodic face; in split
//     coordinates each neighbour cell is a piece of its own);
//   - sources are staged through LDS in tiles of kTile with their periodic
//     image shift applied, then read back by broadcast;
//   - when a cell holds few targets the 64 lanes are split into S groups that
//     take disjoint slices of a tile, and the groups' sums are added in a
//     fixed order through LDS at the end;
//   - a lane may hold two targets, so that every source it reads serves both:
//     an item takes whichever of one or two targets per lane leaves fewer
//     lanes idle (up to 128 targets per item);
//   - the pair loop is plain float32 VALU: one reciprocal square root,
//     the polynomial in registers, the cutoff as a select (Sec. 3.1 describes
//     the same select-based filtering inside the force loop).
// Periodic images are made exact: a target in the last cell layer of an axis
// works in a frame shifted by -L there, so every image shift is 0 or -L and is
// only ever applied to coordinates >= L/2, where subtracting L is exact.
//
// Everything runs on a batch of boxes (one box = a batch of one): a work item
// carries its box, whose geometry, inputs and outputs it reads from the
// batch descriptor.  Items may be ordered by decreasing cost bucket (longest
// first) and are either one workgroup each (a workgroup also takes positions
// + k gridDim when sub-items outnumber the grid) or pulled from a counter by
// persistent workgroups; the sub-items' partial sums are then added by
// k_subsum.
#include <climits>
#include <cmath>

#include "sr_internal.h"
#include "sr_pair.h"

namespace {


// The pair loop of one work item by one wavefront (tile, st, red: LDS).
__device__ __forceinline__ void process_item(const Batch &B, const int4 item,
                                             const float4 *__restrict__ sorted,
                                             const int *__restrict__ offsets,
                                             const int *__restrict__ perm,
                                             const int *__restrict__ mass_mixed,
                                             const ForceParams &fp, float4 *tile, Stencil &st,
                                             int lane, float4 *__restrict__ subsums)
{
    const int kb = item.y, nt = item.z, S = item_split(item), box = item_box(item);
    const BoxDesc &d = box_at(B, box);
    const Geom &g = d.g;
    int cx, cy, cz;
    decode_cell(item.x - d.cbase, g, cx, cy, cz);
    const int cc[3] = {cx, cy, cz};
    float F[3];
    frame_shift(g, cc, F);
    build_stencil(st, offsets + d.cbase, g, cx, cy, cz, F, lane);

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
    const bool uniform = mass_mixed[box] == 0;
    __syncthreads();

    float acx = 0.f, acy = 0.f, acz = 0.f;
    float bcx = 0.f, bcy = 0.f, bcz = 0.f;
    if (__any((has_target && !pas) || (has2 && !pas2))) {
        // a sub-item takes its part [sk T / ns, (sk + 1) T / ns) of the T sources
        const int ns = item_nsub(item), sk = item_sub(item);
        const int all = st.pbeg[kMaxPieces];
        const int total = ns > 1 ? (int)((long long)(sk + 1) * all / ns) : all;
        // a pass stages `cap` sources (a multiple of the 4 S slice quantum, so
        // that padding stays inside the tile); the next pass's sources are
        // loaded before the current pass computes (each load waits for its
        // image shift: deferring the shifts past the pair loop costs this
        // kernel its occupancy step)
        const int quantum = 4 * S;
        const int cap = kItemTab.cap[S];
        const int qrecip = kItemTab.qrecip[S];
        // sources outside the cutoff of the whole box of the item's targets
        // are dropped before they reach the tile
        const TargetBox tb = target_box(xi, yi, zi, xj, yj, zj);
        float4 pre[kTile / 64];
        int p = 0;
        int g0 = ns > 1 ? (int)((long long)sk * all / ns) : 0;
        int cnt = total - g0 < cap ? total - g0 : cap;
        load_tile(pre, st, sorted, g0, cnt, lane, p);
        for (;;) {
            // kept sources, rounded up to the quantum with entries that add zero
            const int nq = quanta_of(store_tile_kept(tile, pre, tb, fp, lane), quantum, qrecip);
            __syncthreads();
            const int g1 = g0 + cnt;
            const int cnt1 = total - g1 < cap ? total - g1 : cap;
            if (cnt1 > 0)
                load_tile(pre, st, sorted, g1, cnt1, lane, p);
            const int slice = 4 * nq;
            const float4 *src = tile + (has_target ? part : 0) * slice;
            float tx = 0.f, ty = 0.f, tz = 0.f;
            if (two) {
                float ux = 0.f, uy = 0.f, uz = 0.f;
                if (uniform)
                    pair_tile2<true>(src, slice, xi, yi, zi, xj, yj, zj, fp, tx, ty, tz, ux, uy,
                                     uz);
                else
                    pair_tile2<false>(src, slice, xi, yi, zi, xj, yj, zj, fp, tx, ty, tz, ux, uy,
                                      uz);
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
        if (uniform) {
            acx *= pt.w;
            acy *= pt.w;
            acz *= pt.w;
            bcx *= pt2.w;
            bcy *= pt2.w;
            bcz *= pt2.w;
        }
    }
    // add the S group sums of each target in group order
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
        // sub-item 0 writes the accelerations as a whole item does, sub-item
        // sk > 0 its partial sums to plane sk - 1
        const int sub = item_sub(item);
        float4 *pp = sub > 0 ? subsums + (size_t)(sub - 1) * B.ntot : nullptr;
        if (pp) {
            pp[kb + t] = pas ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(acx, acy, acz, 0.f);
        } else {
            const int orig = perm[kb + t] - d.pbase;
            d.ax[orig] = pas ? 0.f : acx;
            d.ay[orig] = pas ? 0.f : acy;
            d.az[orig] = pas ? 0.f : acz;
        }
        if (has2) {
            for (int q = 1; q < S; ++q) {
                const float4 o = tile[64 + t + q * ln];
                bcx += o.x;
                bcy += o.y;
                bcz += o.z;
            }
            if (pp) {
                pp[kb + t + ln] =
                    pas2 ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(bcx, bcy, bcz, 0.f);
            } else {
                const int orig2 = perm[kb + t + ln] - d.pbase;
                d.ax[orig2] = pas2 ? 0.f : bcx;
                d.ay[orig2] = pas2 ? 0.f : bcy;
                d.az[orig2] = pas2 ? 0.f : bcz;
            }
        }
    }
    __syncthreads();  // the tile is reused by the next item
}

// Position in the item order served by workgroup b: workgroups are dealt to
// the 8 XCDs round-robin, and XCD k serves the chunks of 64 consecutive
// items k, k + 8, k + 16, ..., so each XCD sees the same mix of costs and
// neighbouring cells (shared sources) meet in one L2.  A bijection on
// [0, grid) for grid a multiple of 512.
__device__ __forceinline__ int item_position(int b)
{
    const int xcd = b & 7, j = b >> 3;
    return ((j >> 6) * 8 + xcd) * 64 + (j & 63);
}

// One workgroup per item: the grid covers the chunk bound (a multiple of 512;
// at most kMaskedGrid workgroups in masked passes), and a workgroup also
// serves positions + k gridDim when sub-items make more items than that.
__global__ __launch_bounds__(64) void k_force(Batch B, const int4 *__restrict__ items,
                                              const int *__restrict__ n_items,
                                              const float4 *__restrict__ sorted,
                                              const int *__restrict__ offsets,
                                              const int *__restrict__ perm,
                                              const int *__restrict__ mass_mixed, ForceParams fp,
                                              float4 *__restrict__ subsums)
{
    __shared__ float4 tile[kTile];
    __shared__ Stencil st;
    const int n = *n_items;
    for (int pos = item_position(blockIdx.x); pos < n; pos += gridDim.x)
        process_item(B, items[pos], sorted, offsets, perm, mass_mixed, fp, tile, st, threadIdx.x,
                     subsums);
}

// Adds the partial sums of the sub-items of every chunk cut into sub-items
// (heads: each chunk's first sub-item), in sub-item order -- sub-item 0's
// sums are in the outputs already -- and writes the chunk's accelerations
// (passive targets' partials are exact zeros).
// Thread g of the grid-stride loop takes target g % kChunk2 of head g / kChunk2.
__global__ __launch_bounds__(256) void k_subsum(Batch B, const int4 *__restrict__ heads,
                                                const int *__restrict__ n_heads,
                                                const int *__restrict__ perm,
                                                const float4 *__restrict__ subsums)
{
    const long long n = (long long)*n_heads * kChunk2;
    for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < n;
         g += (long long)gridDim.x * 256) {
        const int4 item = heads[g / kChunk2];
        const int t = (int)(g % kChunk2);
        const int ns = item_nsub(item);
        const BoxDesc &d = box_at(B, item_box(item));
        if (t < item.z) {
            const int slot = item.y + t;
            const int orig = perm[slot] - d.pbase;
            float ax = d.ax[orig], ay = d.ay[orig], az = d.az[orig];
            for (int k = 1; k < ns; ++k) {
                const float4 v = subsums[(size_t)(k - 1) * B.ntot + slot];
                ax += v.x;
                ay += v.y;
                az += v.z;
            }
            d.ax[orig] = ax;
            d.ay[orig] = ay;
            d.az[orig] = az;
        }
    }
}

// Persistent variant: a fixed grid of workgroups takes kPersistentGrab
// consecutive items at a time from a counter until none are left (every
// workgroup reaches the exit).  Taking two per atomic halves the traffic on
// the one counter address, which bounded the pass on many-item batches.
constexpr int kPersistentGrab = 2;
__global__ __launch_bounds__(64) void k_force_persistent(Batch B, const int4 *__restrict__ items,
                                                         const int *__restrict__ n_items,
                                                         const float4 *__restrict__ sorted,
                                                         const int *__restrict__ offsets,
                                                         const int *__restrict__ perm,
                                                         const int *__restrict__ mass_mixed,
                                                         ForceParams fp, int *__restrict__ queue,
                                                         float4 *__restrict__ subsums)
{
    __shared__ float4 tile[kTile];
    __shared__ Stencil st;
    __shared__ int next;
    const int n = *n_items;
    for (;;) {
        if (threadIdx.x == 0)
            next = atomicAdd(queue, kPersistentGrab);
        __syncthreads();
        const int p0 = next;
        __syncthreads();
        if (p0 >= n)
            break;
        const int pe = p0 + kPersistentGrab < n ? p0 + kPersistentGrab : n;
        for (int pos = p0; pos < pe; ++pos)
            process_item(B, items[pos], sorted, offsets, perm, mass_mixed, fp, tile, st,
                         threadIdx.x, subsums);
    }
}

// Useful-pair and candidate counts with the same stencil and cutoff test
// (one box).
__global__ __launch_bounds__(64) void k_pair_stats(Batch B, const int4 *__restrict__ items,
                                                   const int *__restrict__ n_items,
                                                   const float4 *__restrict__ sorted,
                                                   const int *__restrict__ offsets,
                                                   const int *__restrict__ perm, ForceParams fp,
                                                   int *__restrict__ per_target,
                                                   unsigned long long *__restrict__ stats)
{
    __shared__ float4 tile[kTile];
    __shared__ Stencil st;
    const int lane = threadIdx.x;
    const int it = blockIdx.x;
    if (it >= *n_items)
        return;
    const int4 item = items[it];
    const int kb = item.y, nt = item.z;
    const BoxDesc &d = box_at(B, item_box(item));
    const Geom &g = d.g;
    int cx, cy, cz;
    decode_cell(item.x - d.cbase, g, cx, cy, cz);
    const int cc[3] = {cx, cy, cz};
    float F[3];
    frame_shift(g, cc, F);
    build_stencil(st, offsets + d.cbase, g, cx, cy, cz, F, lane);
    // up to 128 targets: lane l counts for targets l and l + 64
    bool act[2], has[2];
    float xi[2], yi[2], zi[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        has[h] = lane + 64 * h < nt;
        const float4 pt = sorted[kb + (has[h] ? lane + 64 * h : 0)];
        act[h] = has[h] && !is_passive(pt, g);
        xi[h] = pt.x + F[0];
        yi[h] = pt.y + F[1];
        zi[h] = pt.z + F[2];
    }
    __syncthreads();
    const int total = st.pbeg[kMaxPieces];
    // the force pass's box test, so that the counts cover exactly the sources
    // it evaluates (and a useful pair it dropped would show in per_target)
    const TargetBox tb = target_box(xi[0], yi[0], zi[0], xi[1], yi[1], zi[1]);
    int cntu[2] = {0, 0};
    int kept = 0;
    int p = 0;
    for (int g0 = 0; g0 < total; g0 += kTile) {
        const int cnt = total - g0 < kTile ? total - g0 : kTile;
        float4 pre[kTile / 64];
        load_tile(pre, st, sorted, g0, cnt, lane, p);
        const int nk = store_tile_kept(tile, pre, tb, fp, lane);
        kept += nk;
        __syncthreads();
        for (int j = 0; j < nk; ++j) {
            const float4 s = tile[j];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float dx = s.x - xi[h], dy = s.y - yi[h], dz = s.z - zi[h];
                const float se = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, fp.eps)));
                cntu[h] += se < fp.rcut ? 1 : 0;
            }
        }
        __syncthreads();
    }
    unsigned long long u = 0ull, c = 0ull;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cntu[h] = act[h] ? cntu[h] - 1 : 0;  // the target itself is always in its stencil
        if (has[h] && per_target)
            per_target[perm[kb + lane + 64 * h] - d.pbase] = cntu[h];
        u += (unsigned long long)cntu[h];
        c += act[h] ? (unsigned long long)kept : 0ull;
    }
    for (int o = 1; o < 64; o <<= 1) {
        u += __shfl_xor(u, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if (lane == 0) {
        atomicAdd(&stats[0], u);
        atomicAdd(&stats[1], c);
    }
}

// Work items of a block of 256 cells: each thread takes one cell's chunk
// count and stencil size (cells flagged kFineFlag are chunked here: long
// chunks cut into sub-items, short ones finer; with split, the chunks of
// boxes that box_splits admits are cut into sub-items by their pair count;
// with target counts, a masked pass, the chunks cover the cell's first
// tcount[c] slots, where its active particles sit), the block
// reserves its item range with one atomic on *n_items, then all threads
// write the block's items, thread j the items j, j + 256, ... (the cell of an
// item found by a binary search over the block's running item counts).  The
// order of the items depends on which block reserves first; no result does:
// every target is summed in a fixed order, by one item or by its chunk's
// sub-items added in order.  The first sub-item of every cut chunk is also
// appended to heads, for k_subsum.
__global__ __launch_bounds__(256) void k_items(Batch B, const int *__restrict__ offsets,
                                               const int *__restrict__ chunk_count,
                                               const int *__restrict__ tcount, int split,
                                               int4 *__restrict__ items,
                                               int *__restrict__ item_cost,
                                               int *__restrict__ n_items,
                                               int4 *__restrict__ heads,
                                               int *__restrict__ n_heads)
{
    __shared__ int wsum[4];
    __shared__ int base;
    __shared__ int s_end[256];  // the block's items up to and including each cell
    __shared__ int s_q[256], s_ns[256], s_b[256], s_len[256], s_box[256];
    __shared__ long long s_src[256];
    __shared__ bool s_mesh[256];  // chunks laid out as mesh_chunks lays them out, or equal
    const int c = blockIdx.x * 256 + threadIdx.x;
    // masked passes: the counts binning left; otherwise the cell's chunks
    const int cc = c >= B.ctot ? 0
                   : tcount    ? chunk_count[c]
                               : mesh_chunks(offsets[c + 1] - offsets[c]);
    const bool fine = (cc & kFineFlag) != 0;
    int q = cc & (kFineFlag - 1);
    int ns = 1, box = 0, b = 0, len = 0;
    bool mesh = true;
    long long src = 0;
    if (q > 0 || fine) {
        src = cell_stencil(B, offsets, c, &box, &b, &len);
        if (tcount)
            len = tcount[c];  // the active particles, sorted to the front of the cell
        long long k = 1;
        if (fine) {
            // long chunks (dense cells): whole chunks cut into sub-items by
            // their pair count; short ones: chunks of at most kFineChunk
            // targets cut by their source count, so that passes over few
            // cells still have many items
            const int qm = mesh_chunks(len);
            const long long pm = src * ((len + qm - 1) / qm);
            const bool whole = pm > kSplitPairs;
            mesh = whole;
            q = whole ? qm : (len + kFineChunk - 1) / kFineChunk;
            k = whole ? (pm + kSplitPairs - 1) / kSplitPairs
                      : (src + kFineSources - 1) / kFineSources;
        } else if (split && box_splits(box_at(B, box).n)) {
            k = (src * ((len + q - 1) / q) + kSplitPairs - 1) / kSplitPairs;
        }
        ns = k < 1 ? 1 : (k > kMaxSrcSplit ? kMaxSrcSplit : (int)k);
    }
    const int m = q * ns;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int tot;
    int first = wave_exclusive_scan(m, lane, &tot);
    if (lane == 0)
        wsum[wid] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        base = t > 0 ? atomicAdd(n_items, t) : 0;
    }
    for (int j = 0; j < wid; ++j)
        first += wsum[j];
    s_end[threadIdx.x] = first + m;
    s_q[threadIdx.x] = q;
    s_ns[threadIdx.x] = ns;
    s_b[threadIdx.x] = b;
    s_len[threadIdx.x] = len;
    s_box[threadIdx.x] = box;
    s_src[threadIdx.x] = src;
    s_mesh[threadIdx.x] = mesh;
    __syncthreads();
    const int T = s_end[255];
    for (int j = threadIdx.x; j < T; j += 256) {
        int lo = 0, hi = 255;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s_end[mid] > j)
                hi = mid;
            else
                lo = mid + 1;
        }
        const int qq = s_q[lo], nn = s_ns[lo];
        const int r = j - (s_end[lo] - qq * nn);
        const int k = r / nn;
        int bucket;
        const int4 it = cell_item(blockIdx.x * 256 + lo, s_box[lo], s_b[lo], s_len[lo], qq,
                                  s_mesh[lo], k, nn, r - k * nn, s_src[lo], &bucket);
        items[base + j] = it;
        item_cost[base + j] = bucket;
        if (nn > 1 && r == k * nn)
            heads[atomicAdd(n_heads, 1)] = it;
    }
}

// Longest-first order of the items: a counting sort by decreasing cost
// bucket (key = 31 - bucket).  k_lpt_hist adds every block's key counts into
// 32 global totals; k_lpt_scatter gives key k the range starting at the
// totals of the keys before it, reserves one sub-range per (block, key) with
// an atomic, and places its items there in their original order.  Which
// block gets which sub-range depends on timing, so the item order inside a
// key is not fixed -- results are: every target is summed entirely inside
// one item, in a fixed order, whatever the order of the items.
// lpt[0..31] are the key totals and lpt[32..63] the key cursors, both zero
// on entry (the binning pass clears them).
__global__ __launch_bounds__(256) void k_lpt_hist(const int *__restrict__ item_cost,
                                                  const int *__restrict__ n_items,
                                                  int *__restrict__ lpt)
{
    __shared__ int h[32];
    if (threadIdx.x < 32)
        h[threadIdx.x] = 0;
    __syncthreads();
    const int n = *n_items;
    for (int k = 0; k < kLptBlock / 256; ++k) {
        const int i = blockIdx.x * kLptBlock + k * 256 + threadIdx.x;
        if (i < n)
            atomicAdd(&h[31 - item_cost[i]], 1);
    }
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x] > 0)
        atomicAdd(&lpt[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void k_lpt_scatter(const int4 *__restrict__ items,
                                                     const int *__restrict__ item_cost,
                                                     const int *__restrict__ n_items,
                                                     int *__restrict__ lpt,
                                                     int4 *__restrict__ out)
{
    __shared__ int run[32];
    __shared__ int hcnt[32];
    __shared__ int wcnt[4][32];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int n = *n_items;
    if ((int)blockIdx.x * kLptBlock >= n)
        return;
    if (threadIdx.x < 32)
        hcnt[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < kLptBlock / 256; ++k) {
        const int i = blockIdx.x * kLptBlock + k * 256 + threadIdx.x;
        if (i < n)
            atomicAdd(&hcnt[31 - item_cost[i]], 1);
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        int base = 0;
        for (int k = 0; k < (int)threadIdx.x; ++k)
            base += lpt[k];
        const int c = hcnt[threadIdx.x];
        run[threadIdx.x] = c > 0 ? base + atomicAdd(&lpt[32 + threadIdx.x], c) : 0;
    }
    for (int k = 0; k < kLptBlock / 256; ++k) {
        if (threadIdx.x < 128)
            wcnt[threadIdx.x >> 5][threadIdx.x & 31] = 0;
        __syncthreads();
        const int i = blockIdx.x * kLptBlock + k * 256 + threadIdx.x;
        const bool live = i < n;
        const int key = live ? 31 - item_cost[i] : 0;
        // lanes of this wavefront with the same key, by 5 ballots
        unsigned long long same = __ballot(live);
#pragma unroll
        for (int bit = 0; bit < 5; ++bit) {
            const unsigned long long v = __ballot(live && ((key >> bit) & 1));
            same &= ((key >> bit) & 1) ? v : ~v;
        }
        const int rank = __popcll(same & ((1ull << lane) - 1ull));
        if (live && rank == 0)
            wcnt[wid][key] = __popcll(same);
        __syncthreads();
        if (live) {
            int before = run[key];
            for (int w = 0; w < wid; ++w)
                before += wcnt[w][key];
            out[before + rank] = items[i];
        }
        __syncthreads();
        if (threadIdx.x < 32)
            run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] +
                                wcnt[2][threadIdx.x] + wcnt[3][threadIdx.x];
        __syncthreads();
    }
}

// FP64 sum_i m_i a_i per box.  Box b is cut into R_b = min(kRedBlocks,
// ceil(n_b / 4096)) contiguous chunks, one per block; within a block each
// thread sums a fixed strided subset and the block adds them in a fixed tree
// order.  Blocks past R_b contribute exact zeros, so a box's sum depends on
// that box alone (bitwise the same alone and in a batch).
__global__ __launch_bounds__(256) void k_momentum_partial(Batch B, double *__restrict__ part)
{
    __shared__ double sh[3][256];
    const BoxDesc &d = box_at(B, blockIdx.y);
    int R = (d.n + 4095) / 4096;
    R = R < 1 ? 1 : (R > kRedBlocks ? kRedBlocks : R);
    const int chunk = (d.n + R - 1) / R;
    const int lo = blockIdx.x * chunk;
    const int hi = (int)blockIdx.x < R ? (lo + chunk < d.n ? lo + chunk : d.n) : lo;
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = lo + threadIdx.x; i < hi; i += 256) {
        const double mi = (double)d.m[i];
        s[0] += mi * (double)d.ax[i];
        s[1] += mi * (double)d.ay[i];
        s[2] += mi * (double)d.az[i];
    }
    for (int k = 0; k < 3; ++k)
        sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k)
                sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k)
            part[(blockIdx.y * kRedBlocks + blockIdx.x) * 3 + k] = sh[k][0];
}

// One block per box: the kRedBlocks partials added in a fixed tree order.
__global__ __launch_bounds__(256) void k_momentum_final(const double *__restrict__ part,
                                                        double *__restrict__ out)
{
    __shared__ double sh[3][256];
    for (int k = 0; k < 3; ++k) {
        double v = 0.0;
        for (int r = threadIdx.x; r < kRedBlocks; r += 256)
            v += part[(blockIdx.x * kRedBlocks + r) * 3 + k];
        sh[k][threadIdx.x] = v;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k)
                sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3)
        out[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

constexpr unsigned kMaskedGrid = 65536;  // workgroups of a masked pass at most (a multiple of 512)
constexpr unsigned kSubsumGrid = 256;    // workgroups of k_subsum (256 threads each)

unsigned grid_for_items(int64_t ub)
{
    return (unsigned)((ub + 511) & ~int64_t(511));
}

int lpt_blocks(int64_t ub)
{
    return (int)((ub + kLptBlock - 1) / kLptBlock);
}

}  // namespace

int64_t item_bound(int64_t ntot, int64_t ctot, bool split)
{
    int64_t nonempty = ntot < ctot ? ntot : ctot;
    // at most max(ceil(n / 64), n / 16) <= n / 16 + 1 chunks per cell
    // (mesh_chunks_for; flagged cells take ceil(n / kFineChunk) <= n / 32 + 1),
    // each of at most kMaxSrcSplit sub-items when chunks may be cut
    const int64_t chunks = nonempty + ntot / 16 + 1;
    return split ? kMaxSrcSplit * chunks : chunks;
}

void force_layout(Bump &b, int64_t ntot, int64_t ctot, int nb, ForceScratch &s, bool masked,
                  bool split_ok)
{
    size_t nn = (size_t)(ntot > 0 ? ntot : 1);
    const bool split = masked || split_ok;
    const int64_t ub = item_bound(ntot, ctot, split);
    bin_layout(b, ntot, ctot, nb, s.bin);
    s.offsets = b.take<int>((size_t)ctot + 1);
    s.perm = b.take<int>(nn);
    s.sorted = b.take<float4>(nn);
    s.chunk_count = b.take<int>((size_t)ctot);
    s.items = b.take<int4>((size_t)ub);
    s.item_cost = b.take<int>((size_t)ub);
    s.items_lpt = b.take<int4>((size_t)ub);
    s.queue = b.take<int>(1);
    s.mom_part = b.take<double>((size_t)(nb > 0 ? nb : 1) * kRedBlocks * 3);
    s.part = split ? b.take<float4>(nn * (kMaxSrcSplit - 1)) : nullptr;
    s.heads = split ? b.take<int4>((size_t)item_bound(ntot, ctot)) : nullptr;
    s.tcount = masked ? b.take<int>((size_t)ctot) : nullptr;
}

int check_force_params(sr_ctx *ctx, float r_max, float eps, const float *poly)
{
    if (!poly)
        return sr_fail(ctx, SR_EINVAL, "poly is NULL");
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(poly[k]))
            return sr_fail(ctx, SR_EINVAL, "poly[%d] is not finite", k);
    if (!(r_max > 0.f) || !std::isfinite(r_max))
        return sr_fail(ctx, SR_EINVAL, "r_max must be > 0");
    if (!(eps >= 1e-20f) || !std::isfinite(eps))
        return sr_fail(ctx, SR_EINVAL,
                       "eps must be >= 1e-20 (a pair at zero distance must stay finite)");
    return SR_OK;
}

// Validates one box against the cutoff and returns the pair loop's geometry.
int check_box_args(sr_ctx *ctx, const sr_box *box, double cell, float r_max, int xsplit, Geom *g)
{
    int rc = sr_make_geom(ctx, box, cell, g);
    if (rc)
        return rc;
    for (int d = 0; d < 3; ++d) {
        double cs = g->len[d] / g->nc[d];  // chaining cell width
        if ((double)r_max > cs)
            return sr_fail(ctx, SR_EINVAL,
                           "r_max=%g exceeds the cell width %g on axis %d: 27 cells would not "
                           "cover the cutoff",
                           (double)r_max, cs, d);
        if (g->periodic && g->nc[d] < 3)
            return sr_fail(ctx, SR_EINVAL,
                           "periodic box needs >= 3 cells per axis (axis %d has %d)", d,
                           g->nc[d]);
        if (g->periodic && !(2.0 * (double)r_max < g->len[d]))
            return sr_fail(ctx, SR_EINVAL, "periodic box needs 2 r_max < L");
    }
    return sr_make_geom(ctx, box, cell, g, xsplit);
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

int lpt_sort_enqueue(sr_ctx *ctx, const int4 *items, const int *item_cost, const int *n_items,
                     int64_t bound, int *lpt, int4 *out)
{
    const int nblk = lpt_blocks(bound);
    hipLaunchKernelGGL(k_lpt_hist, dim3(nblk), dim3(256), 0, ctx->stream, item_cost, n_items, lpt);
    hipLaunchKernelGGL(k_lpt_scatter, dim3(nblk), dim3(256), 0, ctx->stream, items, item_cost,
                       n_items, lpt, out);
    return sr_check_launch(ctx, "k_lpt");
}

// Binning with the per-cell item counts, the work items, then the
// longest-first order when asked for.
static int bin_items_enqueue(sr_ctx *ctx, const Batch &B, const ForceScratch &s, int order)
{
    int rc;
    if ((rc = bin_enqueue(ctx, B, s.bin, s.offsets, s.perm, s.sorted, s.chunk_count, s.tcount)))
        return rc;
    hipLaunchKernelGGL(k_items, dim3((B.ctot + 255) / 256), dim3(256), 0, ctx->stream, B,
                       s.offsets, s.chunk_count, s.tcount, s.part != nullptr ? 1 : 0, s.items,
                       s.item_cost, s.bin.n_items, s.heads, s.bin.n_heads);
    if ((rc = sr_check_launch(ctx, "k_items")))
        return rc;
    if (order == 1)
        return lpt_sort_enqueue(ctx, s.items, s.item_cost, s.bin.n_items,
                                item_bound(B.ntot, B.ctot, s.part != nullptr), s.bin.lpt,
                                s.items_lpt);
    return SR_OK;
}

int force_enqueue(sr_ctx *ctx, const Batch &B, const ForceScratch &s, const ForceParams &fp,
                  int order, int persistent, double *mom, int rec)
{
    int rc;
    sr_timing_mark(ctx, rec, 0);
    if ((rc = bin_items_enqueue(ctx, B, s, order)))
        return rc;
    sr_timing_mark(ctx, rec, 1);
    const int4 *items = order == 1 ? s.items_lpt : s.items;
    const int *n_items = s.bin.n_items;
    if (B.ntot > 0) {
        if (persistent) {
            int dev_cus = 256;
            (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount,
                                        ctx->device);
            const int64_t ub = item_bound(B.ntot, B.ctot);
            int64_t grid = (int64_t)dev_cus * 24;
            if (grid > ub)
                grid = ub;
            if ((rc = fill_enqueue(ctx, s.queue, 0, 1)))
                return rc;
            hipLaunchKernelGGL(k_force_persistent, dim3((unsigned)grid), dim3(64), 0, ctx->stream,
                               B, items, n_items, s.sorted, s.offsets, s.perm, s.bin.mass_mixed,
                               fp, s.queue, s.part);
        } else {
            // with sub-items the item bound is loose: the grid covers the
            // chunk bound (at most kMaskedGrid workgroups in masked passes,
            // which have few items) and walks the rest
            unsigned grid = grid_for_items(item_bound(B.ntot, B.ctot));
            if (s.tcount && grid > kMaskedGrid)
                grid = kMaskedGrid;
            hipLaunchKernelGGL(k_force, dim3(grid), dim3(64), 0, ctx->stream, B, items, n_items,
                               s.sorted, s.offsets, s.perm, s.bin.mass_mixed, fp, s.part);
        }
        if ((rc = sr_check_launch(ctx, "k_force")))
            return rc;
        // the sub-items' partial sums, added in order
        if (s.part) {
            hipLaunchKernelGGL(k_subsum, dim3(kSubsumGrid), dim3(256), 0, ctx->stream, B,
                               s.heads, s.bin.n_heads, s.perm, s.part);
            if ((rc = sr_check_launch(ctx, "k_subsum")))
                return rc;
        }
    }
    sr_timing_mark(ctx, rec, 2);
    if (mom) {
        hipLaunchKernelGGL(k_momentum_partial, dim3(kRedBlocks, B.nb), dim3(256), 0, ctx->stream,
                           B, s.mom_part);
        hipLaunchKernelGGL(k_momentum_final, dim3(B.nb), dim3(256), 0, ctx->stream, s.mom_part,
                           mom);
        if ((rc = sr_check_launch(ctx, "k_momentum")))
            return rc;
    }
    return SR_OK;
}

int momentum_enqueue(sr_ctx *ctx, const Batch &B, double *part, double *mom)
{
    hipLaunchKernelGGL(k_momentum_partial, dim3(kRedBlocks, B.nb), dim3(256), 0, ctx->stream, B,
                       part);
    hipLaunchKernelGGL(k_momentum_final, dim3(B.nb), dim3(256), 0, ctx->stream, part, mom);
    return sr_check_launch(ctx, "k_momentum");
}

// Batch of one box, by value.
int single_batch(sr_ctx *ctx, const float *x, const float *y, const float *z,
                        const float *mass, int64_t n, const sr_box *box, double cell, float r_max,
                        int xsplit, float *ax, float *ay, float *az, Batch *B)
{
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n=%lld out of range", (long long)n);
    if (n > 0 && (!x || !y || !z))
        return sr_fail(ctx, SR_EINVAL, "NULL coordinate pointer");
    *B = Batch{};
    int rc = check_box_args(ctx, box, cell, r_max, xsplit, &B->one.g);
    if (rc)
        return rc;
    B->nb = 1;
    B->ntot = (int)n;
    B->ctot = B->one.g.ncell;
    B->one.n = (int)n;
    B->one.x = x;
    B->one.y = y;
    B->one.z = z;
    B->one.m = mass;
    B->one.ax = ax;
    B->one.ay = ay;
    B->one.az = az;
    return SR_OK;
}

// sr_force_split with an optional activity mask (cells without an active
// particle get no work items; their particles' outputs are left as they
// were).  Also the arena bytes such a call uses (bytes != nullptr: sizing
// only, nothing is enqueued).
int force_split_masked(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                       const float *oz, const float *mass, int64_t n, const sr_box *box,
                       double cell, float r_max, float eps, const float poly[6], float *ax,
                       float *ay, float *az, double *momentum3, const unsigned char *active,
                       size_t *bytes)
{
    int rc = check_force_params(ctx, r_max, eps, poly);
    if (rc)
        return rc;
    if (!box || !box->periodic)
        return sr_fail(ctx, SR_EINVAL, "split coordinates need a periodic box");
    const int xs = ctx->xsplit < 3 ? ctx->xsplit : 3;
    Batch B;
    if ((rc = single_batch(ctx, ox, oy, oz, mass, n, box, cell, r_max, xs, ax, ay, az, &B)))
        return rc;
    if (n > 0 && (!cell3 || !mass || !ax || !ay || !az))
        return sr_fail(ctx, SR_EINVAL, "NULL pointer");
    for (int d = 0; d < 3; ++d)
        if (B.one.g.nc[d] / (d == 0 ? xs : 1) > kSplitMaxCells)
            return sr_fail(ctx, SR_EINVAL, "split coordinates allow at most %d cells per axis",
                           kSplitMaxCells);
    B.one.g.split = 1;
    B.one.cell3 = cell3;
    B.one.active = active;
    Bump sz{nullptr, 0, 0};
    ForceScratch s;
    const bool masked = active != nullptr;
    force_layout(sz, n, B.ctot, 1, s, masked, box_splits(n));
    if (bytes) {
        *bytes = sz.off;
        return SR_OK;
    }
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    if ((rc = sr_arena_reserve(ctx, sz.off)))
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    force_layout(b, n, B.ctot, 1, s, masked, box_splits(n));
    const ForceParams fp = make_params(r_max, eps, poly);
    const int rec = sr_timing_begin(ctx);
    return force_enqueue(ctx, B, s, fp, ctx->order, ctx->persistent, momentum3, rec);
}

extern "C" int sr_force_split(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                              const float *oz, const float *mass, int64_t n, const sr_box *box,
                              double cell, float r_max, float eps, const float poly[6], float *ax,
                              float *ay, float *az, double *momentum3)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    return force_split_masked(ctx, cell3, ox, oy, oz, mass, n, box, cell, r_max, eps, poly, ax,
                              ay, az, momentum3, nullptr, nullptr);
}

extern "C" int sr_scratch_bytes(const sr_box *box, double cell, int64_t n, int with_force,
                                size_t *bytes)
{
    if (!bytes || n < 0 || n > INT_MAX || with_force < 0 || with_force > 2)
        return SR_EINVAL;
    Geom g;
    // with_force: the largest x split any context may use
    if (sr_make_geom(nullptr, box, cell, &g, with_force ? kMaxXsplit : 1))
        return SR_EINVAL;
    Bump sz{nullptr, 0, 0};
    if (with_force) {
        ForceScratch s;
        force_layout(sz, n, g.ncell, 1, s, with_force == 2, box_splits(n));
        if (with_force == 2) {
            // the multilevel step's levels, activity mask and cell counts
            // (sr_ksk_step lays them out after the force pass)
            Geom g1;
            if (sr_make_geom(nullptr, box, cell, &g1, 1))
                return SR_EINVAL;
            sz.take<unsigned char>((size_t)n);
            sz.take<unsigned char>((size_t)n);
            sz.take<int>((size_t)g1.ncell);
        }
    } else {
        BinScratch s;
        bin_layout(sz, n, g.ncell, 1, s);
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
    int rc = check_force_params(ctx, r_max, eps, poly);
    if (rc)
        return rc;
    Batch B;
    if ((rc = single_batch(ctx, x, y, z, mass, n, box, cell, r_max, ctx->xsplit, ax, ay, az, &B)))
        return rc;
    if (n > 0 && (!mass || !ax || !ay || !az))
        return sr_fail(ctx, SR_EINVAL, "NULL mass or output pointer");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    Bump sz{nullptr, 0, 0};
    ForceScratch s;
    force_layout(sz, n, B.ctot, 1, s, false, box_splits(n));
    if ((rc = sr_arena_reserve(ctx, sz.off)))
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    force_layout(b, n, B.ctot, 1, s, false, box_splits(n));
    const ForceParams fp = make_params(r_max, eps, poly);
    const int rec = sr_timing_begin(ctx);
    return force_enqueue(ctx, B, s, fp, ctx->order, ctx->persistent, momentum3, rec);
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
    Batch B;
    // masses are not needed; the gather reads x in their place
    int rc = single_batch(ctx, x, y, z, x, n, box, cell, r_max, ctx->xsplit, nullptr, nullptr,
                          nullptr, &B);
    if (rc)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    Bump sz{nullptr, 0, 0};
    ForceScratch s;
    force_layout(sz, n, B.ctot, 1, s, false, false);  // whole chunks
    if ((rc = sr_arena_reserve(ctx, sz.off)))
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    force_layout(b, n, B.ctot, 1, s, false, false);
    if ((rc = bin_items_enqueue(ctx, B, s, 0)))
        return rc;
    // eps = 0 so that se = s and the test is s < r_max^2
    ForceParams fp = make_params(r_max, 0.0f, zero_poly);
    unsigned long long *st = (unsigned long long *)ctx->stats;
    if ((rc = fill_enqueue(ctx, (int *)st, 0, 4)))
        return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_pair_stats, dim3((unsigned)item_bound(n, B.ctot)), dim3(64), 0,
                           ctx->stream, B, s.items, s.bin.n_items, s.sorted, s.offsets,
                           s.perm, fp, per_target, st);
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
