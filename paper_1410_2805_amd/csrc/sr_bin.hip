// Chaining-mesh binning on gfx950: cell ids, histogram, exclusive scan,
// scatter and a per-cell ascending sort of original indices.  The result is
// the stable counting sort of the particles by cell (Sec. 2.4 chaining mesh;
// Sec. 2.7 permutation array; Sec. 3.1 fixed bins of the short-range scale).
//
//   k_cellid   cell of each particle in FP64, histogram by atomic increment
//              (the returned old count is an arrival rank, unordered)
//   scan       exclusive prefix sum: tile sums (the last block to finish
//              scans the tile partials), then the per-tile down pass
//   k_scatter  perm[offsets[cell] + rank] = i (grouped by cell, unordered
//              inside a cell)
//   k_segsort  restores stability: the slots of one cell hold that cell's
//              original indices, so sorting them ascending is exactly the
//              stable order.  Four small cells per wavefront, each index
//              ranked among its own cell's; cells up to 1024 by one
//              wavefront (registers, or a wavefront-private LDS bitonic
//              sort); larger cells go to k_segsort_large (one block,
//              LDS-sorted runs merged by rank).  The pass writes the inverse
//              permutation and, for the force pass, the work items per cell.
//   k_gather   the sorted float4 (x, y, z, m) copy, through the inverse.
// All kernels work on a batch of boxes whose particles and cells are numbered
// consecutively; one box is a batch of one.  Passes of 2^22 particles or
// more without an activity mask take a stable LSD radix sort of the cell ids
// instead (k_cellkey, k_radix_*, k_key_offsets): the same offsets and
// permutation without the histogram's global atomics.  A pass with an activity mask
// bins only the cells whose stencil reaches a cell holding an active particle
// (k_relevant): every source of every target, in the same order, with the
// other cells left empty.
#include <climits>

#include "sr_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096 entries per scan tile

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_inclusive_scan(int v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d)
            v += t;
    }
    return v;
}

// Exclusive scan over a 256-thread block; *total receives the block sum.
__device__ int block_exclusive_scan(int v, int *sh /*[5]*/, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = wave_inclusive_scan(v, lane);
    if (lane == 63)
        sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            int t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[kBlock / 64] = run;
    }
    __syncthreads();
    int r = inc - v + sh[wid];
    *total = sh[kBlock / 64];
    __syncthreads();
    return r;
}

__global__ void k_fill(int *__restrict__ p, int value, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = value;
}

constexpr int kCellidPer = 4;                 // particles per thread
constexpr int kCellidBlock = kBlock * kCellidPer;  // 1024 particles per block

__device__ __forceinline__ int particle_cell(const Batch &B, int i, int *status)
{
    const BoxDesc &d = box_at(B, find_box(B.pstart, B.nb, i));
    const int li = i - d.pbase;
    const float p[3] = {d.x[li], d.y[li], d.z[li]};
    const Geom &g = d.g;
    int c[3];
    bool bad = false;
    if (g.split) {
        // chaining cell from cell3; the x sub-cell from the offset
        const int packed = d.cell3[li];
        const int cc[3] = {packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023};
        const int per[3] = {g.hx, 1, 1};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = (double)p[k];
            const int ncc = g.nc[k] / per[k];
            if (!(v >= 0.0 && v <= 1.0001 * g.w[k] * per[k]) || cc[k] >= ncc) {
                bad = true;
                c[k] = 0;
            } else {
                int sub = (int)floor(v * g.inv[k]);
                sub = sub < per[k] - 1 ? sub : per[k] - 1;
                c[k] = cc[k] * per[k] + sub;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double v = (double)p[k];
            if (!(v >= 0.0 && v < g.len[k])) {  // also catches NaN
                bad = true;
                c[k] = 0;
            } else {
                double t = floor(v * g.inv[k]);
                int ci = (int)t;
                c[k] = ci < g.nc[k] - 1 ? ci : g.nc[k] - 1;
            }
        }
    }
    if (bad)
        atomicOr(status, 1);
    return d.cbase + c[0] + g.nc[0] * (c[1] + g.nc[1] * c[2]);
}

constexpr int kPeelMax = 8;    // lane groups of one cell served per wavefront pass
constexpr int kPeelGroup = 4;  // ... while the groups found hold at least this many lanes

// Cell ids and the histogram.  A block takes 1024 particles and first counts
// them per cell in an LDS hash table, then adds each distinct cell's count to
// the global histogram with one atomic; a particle's arrival rank is its
// block's base plus its rank inside the block (ranks are unordered; the
// per-cell sort restores the stable order).  Clustered input puts many lanes
// of a wavefront in one cell, and their LDS atomics on one address would
// serialize: the lanes sharing the lowest remaining lane's cell are found by
// one ballot and served by a single pair of LDS atomics for the whole group,
// repeated while such groups are large; the remaining lanes go one by one.
//
// With an activity mask (kMasked; flag and tcount cleared) the pass also
// leaves in flag[cell] the largest activity value of the cell's particles (1,
// or 2 for cells cut into finer work items; 0: no active particle) and in
// tcount[cell] the number of its active particles.  A block keeps both in one
// LDS word per cell: the active count in the low kActShift bits, the count of
// those with value 2 above them (at most kCellidBlock each).
constexpr int kActShift = 20;
template <bool kMasked>
__global__ __launch_bounds__(kBlock) void k_cellid(Batch B, int *__restrict__ cid,
                                                   int *__restrict__ slot,
                                                   int *__restrict__ count, int *__restrict__ status,
                                                   int *__restrict__ flag, int *__restrict__ tcount)
{
    __shared__ int hkey[kHash];
    __shared__ int hcnt[kHash];
    __shared__ int hflag[kMasked ? kHash : 1];
    for (int h = threadIdx.x; h < kHash; h += kBlock) {
        hkey[h] = -1;
        hcnt[h] = 0;
        if (kMasked)
            hflag[h] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int hs[kCellidPer], rk[kCellidPer], act[kCellidPer];
    const int base = blockIdx.x * kCellidBlock;
#pragma unroll
    for (int k = 0; k < kCellidPer; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        const bool valid = i < B.ntot;
        int id = -1;
        act[k] = 0;
        if (valid) {
            id = particle_cell(B, i, status);
            cid[i] = id;
            if (kMasked) {
                const BoxDesc &d = box_at(B, find_box(B.pstart, B.nb, i));
                act[k] = d.active ? d.active[i - d.pbase] : 1;
            }
        }
        hs[k] = -1;
        rk[k] = 0;
        unsigned long long rem = __ballot(valid);
        const unsigned long long act_b = kMasked ? __ballot(act[k] > 0) : 0ull;
        const unsigned long long fine_b = kMasked ? __ballot(act[k] == 2) : 0ull;
        for (int it = 0; it < kPeelMax && rem; ++it) {
            const int leader = __ffsll((long long)rem) - 1;
            const int key = __builtin_amdgcn_readlane(id, leader);
            const unsigned long long grp = __ballot(id == key) & rem;
            const int gsize = __popcll(grp);
            int hh = 0, hb = 0;
            if (lane == leader) {
                hh = lds_hash_slot(hkey, key);
                hb = atomicAdd(&hcnt[hh], gsize);
                if (kMasked && (act_b & grp))
                    atomicAdd(&hflag[hh], __popcll(act_b & grp) +
                                              (__popcll(fine_b & grp) << kActShift));
            }
            hh = __builtin_amdgcn_readlane(hh, leader);
            hb = __builtin_amdgcn_readlane(hb, leader);
            if ((grp >> lane) & 1ull) {
                hs[k] = hh;
                rk[k] = hb + (int)__builtin_amdgcn_mbcnt_hi(
                                 (unsigned)(grp >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)grp, 0u));
            }
            rem &= ~grp;
            if (gsize < kPeelGroup)
                break;
        }
        if ((rem >> lane) & 1ull) {
            const int h = lds_hash_slot(hkey, id);
            hs[k] = h;
            rk[k] = atomicAdd(&hcnt[h], 1);
            if (kMasked && act[k] > 0)
                atomicAdd(&hflag[h], act[k] == 2 ? 1 + (1 << kActShift) : 1);
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < kHash; h += kBlock) {
        const int c = hcnt[h];
        if (c > 0) {
            if (kMasked && hflag[h] > 0) {
                atomicMax(&flag[hkey[h]], (hflag[h] >> kActShift) > 0 ? 2 : 1);
                atomicAdd(&tcount[hkey[h]], hflag[h] & ((1 << kActShift) - 1));
            }
            hcnt[h] = atomicAdd(&count[hkey[h]], c);  // becomes the block's base
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCellidPer; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        if (hs[k] >= 0)
            slot[i] = hcnt[hs[k]] + rk[k];
    }
}

// Tile sums; the block that finishes last (a device counter, reset by that
// block) scans the tile partials in place.  No block ever waits for another.
__global__ __launch_bounds__(kBlock) void k_scan_up(const int *__restrict__ in, int m,
                                                    int *__restrict__ part, int ntiles,
                                                    int *__restrict__ done)
{
    __shared__ int sh[8];
    __shared__ bool last;
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        s += (base + k < m) ? in[base + k] : 0;
    int total;
    (void)block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = total;
        __threadfence();
        last = atomicAdd(done, 1) == ntiles - 1;
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    int carry = 0;
    for (int b = 0; b < ntiles; b += kBlock) {
        const int i = b + threadIdx.x;
        const int v = i < ntiles ? __hip_atomic_load(&part[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        int tot;
        const int ex = block_exclusive_scan(v, sh, &tot);
        if (i < ntiles)
            part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        *done = 0;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int *__restrict__ in, int m,
                                                      const int *__restrict__ part,
                                                      int *__restrict__ out)
{
    __shared__ int sh[8];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, sh, &total) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m)
            out[base + k] = run;
        run += v[k];
        if (base + k == m - 1)
            out[m] = run;
    }
}

// With an activity mask the slots of active particles take the sort key
// i | INT_MIN, so that the cell sorts put them first (in index order), ahead
// of the inactive ones; the sorts store the plain index (key & INT_MAX).
__global__ __launch_bounds__(kBlock) void k_scatter(const int *__restrict__ cid,
                                                    const int *__restrict__ slot, int n,
                                                    const int *__restrict__ offsets,
                                                    const unsigned char *__restrict__ active,
                                                    int *__restrict__ perm)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int c = cid[i];
    const int o = offsets[c];
    // masked: the particles of cells left empty (k_relevant) take no slot
    if (active && offsets[c + 1] == o)
        return;
    perm[o + slot[i]] = active && active[i] ? (i | INT_MIN) : i;
}

// Masked passes: a cell is binned when its stencil (x +-hx, y and z +-1,
// periodic: masked passes run in split coordinates) reaches a cell flagged
// active (flag[c] > 0, left by k_cellid); the counts of the others are set to
// zero before the scan, so those cells stay empty.  The cells a target's
// stencil reaches are all binned, in the order a full pass gives them, so the
// sums are those of the full pass.
__global__ __launch_bounds__(kBlock) void k_relevant(Geom g, const int *__restrict__ flag,
                                                     int *__restrict__ count)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.ncell || count[c] == 0)
        return;
    const int cz = div_by(c, g.div_m[0], g.div_s[0]);
    const int rem = c - cz * g.nc[0] * g.nc[1];
    const int cy = div_by(rem, g.div_m[1], g.div_s[1]);
    const int cx = rem - cy * g.nc[0];
    for (int dz = -1; dz <= 1; ++dz) {
        int nz = cz + dz;
        nz = nz < 0 ? nz + g.nc[2] : (nz >= g.nc[2] ? nz - g.nc[2] : nz);
        for (int dy = -1; dy <= 1; ++dy) {
            int ny = cy + dy;
            ny = ny < 0 ? ny + g.nc[1] : (ny >= g.nc[1] ? ny - g.nc[1] : ny);
            const int row = g.nc[0] * (ny + g.nc[1] * nz);
            for (int dx = -g.hx; dx <= g.hx; ++dx) {
                int nx = cx + dx;
                nx = nx < 0 ? nx + g.nc[0] : (nx >= g.nc[0] ? nx - g.nc[0] : nx);
                if (flag[row + nx] > 0)
                    return;
            }
        }
    }
    count[c] = 0;
}

__device__ __forceinline__ int bitonic64(int v, int lane)
{
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            int o = __shfl_xor(v, j, 64);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            int mn = v < o ? v : o;
            int mx = v < o ? o : v;
            v = (lower == up) ? mn : mx;
        }
    }
    return v;
}

__device__ __forceinline__ float4 gather_one(const BoxDesc &d, int v)
{
    const int li = v - d.pbase;
    float x = d.x[li];
    if (d.g.split && d.g.hx > 1) {
        // offset from the x sub-cell corner (same sub-cell rule as k_cellid)
        const double o = (double)x;
        int sub = (int)floor(o * d.g.inv[0]);
        sub = sub < d.g.hx - 1 ? sub : d.g.hx - 1;
        sub = sub > 0 ? sub : 0;
        x = (float)(o - (double)sub * d.g.w[0]);
    }
    return make_float4(x, d.y[li], d.z[li], d.m[li]);
}

// Sorted copy by scattering in input order: sorted[inv[i]] = particle i.
// Reads are coalesced; writes land in runs wherever the input keeps
// neighbours together.  Also flags boxes whose masses are not all equal.
__global__ __launch_bounds__(kBlock) void k_gather(Batch B, const int *__restrict__ inv,
                                                   float4 *__restrict__ sorted,
                                                   int *__restrict__ mass_mixed,
                                                   const int *__restrict__ cid,
                                                   const int *__restrict__ offsets)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool mixed = false;
    int box = 0;
    if (i < B.ntot) {
        box = find_box(B.pstart, B.nb, i);
        const BoxDesc &d = box_at(B, box);
        const float4 q = gather_one(d, i);
        // with cid (masked passes) the particles of empty cells have no slot;
        // every mass still decides mass_mixed, as in a full pass
        if (!cid || offsets[cid[i] + 1] != offsets[cid[i]])
            sorted[inv[i]] = q;
        mixed = q.w != d.m[0];
    }
    // one atomic per wavefront for the lanes that share the lowest flagged
    // lane's box (all of them in a single-box pass), one per lane otherwise
    const unsigned long long flagged = __ballot(mixed);
    if (flagged) {
        const int first = __ffsll((long long)flagged) - 1;
        const int b0 = __shfl(box, first);
        const int lane = threadIdx.x & 63;
        if (mixed && (box != b0 || lane == first))
            atomicOr(&mass_mixed[box], 1);
    }
}

constexpr int kMergeSeg = 16;  // merge outputs per thread segment

// One segment of a merge round over runs of w sorted ints (src[0, P), P a
// multiple of 64, runs [p0, p0 + w) and [p0 + w, p0 + 2w) merged in pairs):
// the kMergeSeg outputs from position o (kMergeSeg divides 2w, so the segment
// stays inside one pair).  Merge path: one binary search along the segment's
// diagonal finds how many of its predecessors come from each run, then a
// sequential merge.  Values are distinct except the INT_MAX padding, which
// only the last run holds.
__device__ __forceinline__ void merge_segment(const int *src, int P, int w, int o,
                                              int (&out)[kMergeSeg])
{
    const int p0 = o & ~(2 * w - 1);
    const int d = o - p0;
    const int *A = src + p0;
    const int lenA = P - p0 < w ? P - p0 : w;
    const int *Bv = A + lenA;
    const int lenB = P - p0 - lenA < w ? P - p0 - lenA : w;
    int lo = d - lenB > 0 ? d - lenB : 0;
    int hi = d < lenA ? d : lenA;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (A[m] < Bv[d - 1 - m])
            lo = m + 1;
        else
            hi = m;
    }
    int i = lo, j = d - lo;
    int a = i < lenA ? A[i] : INT_MAX;
    int b = j < lenB ? Bv[j] : INT_MAX;
#pragma unroll
    for (int k = 0; k < kMergeSeg; ++k) {
        const bool take_a = j >= lenB || (i < lenA && a < b);
        out[k] = take_a ? a : b;
        if (take_a) {
            ++i;
            a = i < lenA ? A[i] : INT_MAX;
        } else {
            ++j;
            b = j < lenB ? Bv[j] : INT_MAX;
        }
    }
}

constexpr int kSegGroup = 4;  // consecutive cells per wavefront

// Large cells are listed by size class, class c holding the cells of
// kLargeCell 2^c + 1 .. kLargeCell 2^(c+1) particles (the last class: all
// larger), so that the block sort can take them biggest first.  Class c's
// list has room for every cell of more than kLargeCell 2^c particles of n.
constexpr int kLargeClasses = 8;
__host__ __device__ inline int large_class_cap(int64_t n, int c)
{
    return (int)(n / ((int64_t)kLargeCell << c) + 1);
}
__host__ __device__ inline int large_class_base(int64_t n, int c)
{
    int b = 0;
    for (int k = 0; k < c; ++k)
        b += large_class_cap(n, k);
    return b;
}
__device__ __forceinline__ int large_class(int len)
{
    const int c = 31 - __clz(len - 1) - 10;  // len > kLargeCell = 2^10
    return c < kLargeClasses - 1 ? c : kLargeClasses - 1;
}

// Sorts one cell's slots [b, b + len) by one wavefront (len <= kLargeCell;
// larger cells are queued for k_segsort_large).
__device__ void sort_cell(int cell, int b, int len, int *__restrict__ perm, int *sb,
                          int *__restrict__ large_list, int *__restrict__ large_count,
                          int *__restrict__ inv, int lane, int ntot)
{
    if (len <= 32) {
        // small cell: each index's rank is the number of smaller ones
        const int v = lane < len ? perm[b + lane] : INT_MAX;
        int rank = 0;
        for (int k = 0; k < len; ++k)
            rank += __builtin_amdgcn_readlane(v, k) < v ? 1 : 0;
        if (lane < len) {
            const int u = v & INT_MAX;
            perm[b + rank] = u;
            if (inv)
                inv[u] = b + rank;
        }
    } else if (len <= 64) {
        int v = lane < len ? perm[b + lane] : INT_MAX;
        v = bitonic64(v, lane) & INT_MAX;
        if (lane < len) {
            perm[b + lane] = v;
            if (inv)
                inv[v] = b + lane;
        }
    } else if (len <= kLargeCell) {
        // runs of 64 sorted in registers, then merge rounds in which each
        // lane takes one segment of kMergeSeg outputs (64 kMergeSeg =
        // kLargeCell), held in registers until every lane has read the round
        const int P = (len + 63) & ~63;
        for (int r = 0; r < P; r += 64) {
            int v = r + lane < len ? perm[b + r + lane] : INT_MAX;
            v = bitonic64(v, lane);
            sb[r + lane] = v;
        }
        wave_sync();
        const int o = lane * kMergeSeg;
        for (int w = 64; w < P; w <<= 1) {
            int v[kMergeSeg];
            if (o < P)
                merge_segment(sb, P, w, o, v);
            wave_sync();
            if (o < P) {
#pragma unroll
                for (int k = 0; k < kMergeSeg; ++k)
                    sb[o + k] = v[k];
            }
            wave_sync();
        }
        for (int t = lane; t < len; t += 64) {
            const int v = sb[t] & INT_MAX;
            perm[b + t] = v;
            if (inv)
                inv[v] = b + t;
        }
        wave_sync();
    } else if (lane == 0) {
        const int c = large_class(len);
        const int k = atomicAdd(&large_count[c], 1);
        large_list[large_class_base(ntot, c) + k] = cell;
    }
}

// One wavefront per group of kSegGroup consecutive cells.  When the group
// holds at most 64 particles, each lane takes one slot and ranks its index
// among the smaller indices of the same cell (one pass for the whole group);
// otherwise the cells are sorted one after the other.  With an activity mask
// (chunk_count and tcount), the pass also counts the force work items of
// each cell (mesh_chunks_for).
// Indices are compared as the signed keys k_scatter wrote.
__global__ __launch_bounds__(kBlock) void k_segsort(Batch B, const int *__restrict__ offsets,
                                                    int *__restrict__ perm,
                                                    int *__restrict__ large_list,
                                                    int *__restrict__ large_count,
                                                    int *__restrict__ inv,
                                                    int *__restrict__ chunk_count,
                                                    const int *__restrict__ tcount)
{
    __shared__ int buf[kBlock / 64][kLargeCell];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int c0 = (blockIdx.x * (kBlock / 64) + wid) * kSegGroup;
    if (c0 >= B.ctot)
        return;
    const int nc = B.ctot - c0 < kSegGroup ? B.ctot - c0 : kSegGroup;
    if (chunk_count && tcount && lane < nc) {
        // with an activity mask only the cell's na active particles (sorted
        // first) are targets: cells without one get no item, those flagged 2
        // are marked kFineFlag and cut by k_items (k_cellid left the flags in
        // chunk_count, the counts in tcount)
        const int c = c0 + lane;
        const int f = chunk_count[c], na = tcount[c];
        chunk_count[c] = f == 0 ? 0 : (f >= 2 ? kFineFlag : mesh_chunks(na));
    }
    int bounds[kSegGroup + 1];
#pragma unroll
    for (int k = 0; k <= kSegGroup; ++k)
        bounds[k] = __builtin_amdgcn_readfirstlane(offsets[c0 + (k < nc ? k : nc)]);
    const int b = bounds[0];
    const int total = bounds[kSegGroup] - b;
    if (total <= 64) {
        // my slot, my cell (by the group's inner bounds), my index; the rank
        // of my index among the indices of my own cell only, read from the
        // lanes [cb - b, ce - b) by cross-lane permutes over the longest cell
        const int slot = b + lane;
        int mycell = 0;
#pragma unroll
        for (int k = 1; k < kSegGroup; ++k)
            mycell += slot >= bounds[k] ? 1 : 0;
        const int v = lane < total ? perm[slot] : INT_MAX;
        int cb = bounds[0], ce = bounds[1], maxlen = bounds[1] - bounds[0];
#pragma unroll
        for (int k = 1; k < kSegGroup; ++k) {
            cb = mycell >= k ? bounds[k] : cb;
            ce = mycell >= k ? bounds[k + 1] : ce;
            maxlen = bounds[k + 1] - bounds[k] > maxlen ? bounds[k + 1] - bounds[k] : maxlen;
        }
        const int first = cb - b, len = ce - cb;
        int rank = 0;
#pragma unroll 4
        for (int j = 0; j < maxlen; ++j) {
            const int u = __shfl(v, first + (j < len ? j : 0), 64);
            rank += (j < len && u < v) ? 1 : 0;
        }
        if (lane < total) {
            const int iv = v & INT_MAX;
            perm[cb + rank] = iv;
            if (inv)
                inv[iv] = cb + rank;
        }
        return;
    }
    for (int k = 0; k < nc; ++k)
        sort_cell(c0 + k, bounds[k], bounds[k + 1] - bounds[k], perm, buf[wid], large_list,
                  large_count, inv, lane, B.ntot);
}

constexpr int kLargeBlock = 1024;
constexpr int kMergeIlp = 4;
// indices a block sorts in LDS: 160 KiB less 256 bytes of static LDS
constexpr int kLdsCell = 40896;

// Sorts the indices buf[0, len) of one cell ascending (len <= kLdsCell, whole
// block) and returns where the sorted indices lie (buf, or buf + P when the
// last merge round wrote the second half).  Runs of 64 are sorted in
// registers by bitonic networks, one per wavefront; then merge rounds in
// which each entry's new slot is its offset in its run plus its rank among
// the partner run's entries (a binary search; the indices are distinct).  A
// round writes every entry to its new slot in a second buffer -- the other
// half of LDS when the cell fits twice, else the cell's global scratch `out`,
// read back after the round -- so no entry moves while others still search.
// The tail up to whole runs holds INT_MAX, which sorts last and stays put.
__device__ int *lds_sort_cell(int *buf, int len, int *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int P = (len + 63) & ~63;
    const bool twice = 2 * P <= kLdsCell;
    // a wavefront's 64 lanes hold the whole run (P is a multiple of 64)
    for (int e = threadIdx.x; e < P; e += kLargeBlock) {
        int v = e < len ? buf[e] : INT_MAX;
        v = bitonic64(v, lane);
        buf[e] = v;
        if (twice)
            buf[P + e] = INT_MAX;
    }
    __syncthreads();
    int *src = buf;
    int *dst = twice ? buf + P : out;
    for (int w = 64; w < P; w <<= 1) {
        for (int o = threadIdx.x * kMergeSeg; o < P; o += kLargeBlock * kMergeSeg) {
            int v[kMergeSeg];
            merge_segment(src, P, w, o, v);
            // the global scratch covers the cell's len entries only; the
            // padding (largest) lands past them
#pragma unroll
            for (int k = 0; k < kMergeSeg; ++k)
                if (twice || o + k < len)
                    dst[o + k] = v[k];
        }
        __syncthreads();
        if (twice) {
            int *t = src;
            src = dst;
            dst = t;
        } else {
            for (int e = threadIdx.x; e < len; e += kLargeBlock)
                buf[e] = out[e];
            __syncthreads();
        }
    }
    return src;
}

// Block-level sort of one large cell.  Cells of at most kLdsCell indices are
// sorted entirely in LDS (lds_sort_cell).  Larger ones: LDS-sorted runs of
// kLargeCell, then merge rounds in which every element finds its output slot
// from its rank in the partner run (values are distinct original indices), a
// binary search in global memory; the block is kLargeBlock threads wide so
// that more of those dependent loads are in flight per round.
__global__ __launch_bounds__(kLargeBlock) void k_segsort_large(Batch B,
                                                          const int *__restrict__ offsets,
                                                          int *__restrict__ perm,
                                                          int *__restrict__ tmp,
                                                          const int *__restrict__ large_list,
                                                          int *__restrict__ large_count,
                                                          int *__restrict__ inv)
{
    extern __shared__ int buf[];  // kLdsCell entries
    __shared__ int next;
    int cnt[kLargeClasses];
#pragma unroll
    for (int c = 0; c < kLargeClasses; ++c)
        cnt[c] = large_count[c];
    for (;;) {
        // the next cell, biggest class first (large_count[kLargeClasses] is
        // the work counter)
        if (threadIdx.x == 0)
            next = atomicAdd(&large_count[kLargeClasses], 1);
        __syncthreads();
        int w = next;
        __syncthreads();
        int cell = -1;
        for (int c = kLargeClasses - 1; c >= 0; --c) {
            if (w < cnt[c]) {
                cell = large_list[large_class_base(B.ntot, c) + w];
                break;
            }
            w -= cnt[c];
        }
        if (cell < 0)
            break;
        const int b = offsets[cell];
        const int len = offsets[cell + 1] - b;
        if (len <= kLdsCell) {
            for (int e = threadIdx.x; e < len; e += kLargeBlock)
                buf[e] = perm[b + e];
            const int *sorted_idx = lds_sort_cell(buf, len, tmp + b);
            for (int e = threadIdx.x; e < len; e += kLargeBlock) {
                const int v = sorted_idx[e] & INT_MAX;
                perm[b + e] = v;
                if (inv)
                    inv[v] = b + e;
            }
            __syncthreads();
            continue;
        }
        // 1) sort runs of kLargeCell in LDS (bitonic, whole block)
        for (int r0 = 0; r0 < len; r0 += kLargeCell) {
            int rl = len - r0 < kLargeCell ? len - r0 : kLargeCell;
            for (int t = threadIdx.x; t < kLargeCell; t += kLargeBlock)
                buf[t] = t < rl ? perm[b + r0 + t] : INT_MAX;
            __syncthreads();
            for (int k = 2; k <= kLargeCell; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = threadIdx.x; t < kLargeCell / 2; t += kLargeBlock) {
                        int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                        int l = i + j;
                        bool up = (i & k) == 0;
                        int a = buf[i], c = buf[l];
                        if ((a > c) == up) {
                            buf[i] = c;
                            buf[l] = a;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int t = threadIdx.x; t < rl; t += kLargeBlock)
                perm[b + r0 + t] = buf[t];
            __syncthreads();
        }
        // 2) merge rounds, perm <-> tmp
        int *src = perm + b;
        int *dst = tmp + b;
        for (int w = kLargeCell; w < len; w <<= 1) {
            // kMergeIlp elements per thread; each search step loads for all of
            // them before comparing, so the loads are in flight together
            for (int e0 = threadIdx.x; e0 < len; e0 += kMergeIlp * kLargeBlock) {
                int v[kMergeIlp], lo[kMergeIlp], base[kMergeIlp], cnt[kMergeIlp];
                int at[kMergeIlp];
#pragma unroll
                for (int k = 0; k < kMergeIlp; ++k) {
                    const int e = e0 + k * kLargeBlock;
                    cnt[k] = 0;
                    at[k] = -1;
                    v[k] = 0;
                    lo[k] = 0;
                    base[k] = 0;
                    if (e < len) {
                        const int pair0 = (e / (2 * w)) * (2 * w);
                        const int mid = pair0 + w;  // start of the right run
                        const int end = pair0 + 2 * w < len ? pair0 + 2 * w : len;
                        v[k] = src[e];
                        // left element: count right elements < v, and back
                        const int l = e < mid ? mid : pair0, h = e < mid ? end : mid;
                        lo[k] = l;
                        base[k] = l;
                        cnt[k] = h > l ? h - l : 0;
                        at[k] = pair0 + (e < mid ? e - pair0 : e - mid);
                    }
                }
                for (;;) {
                    int x[kMergeIlp];
                    bool more = false;
#pragma unroll
                    for (int k = 0; k < kMergeIlp; ++k) {
                        // a finished search reads slot 0 of the cell (in range)
                        x[k] = src[cnt[k] > 0 ? base[k] + (cnt[k] >> 1) : 0];
                        more = more || cnt[k] > 0;
                    }
                    if (!more)
                        break;
#pragma unroll
                    for (int k = 0; k < kMergeIlp; ++k) {
                        const int half = cnt[k] >> 1;
                        const bool right = cnt[k] > 0 && x[k] < v[k];
                        base[k] = right ? base[k] + half + 1 : base[k];
                        cnt[k] = cnt[k] > 0 ? (right ? cnt[k] - half - 1 : half) : 0;
                    }
                }
#pragma unroll
                for (int k = 0; k < kMergeIlp; ++k)
                    if (at[k] >= 0)
                        dst[at[k] + (base[k] - lo[k])] = v[k];
            }
            __syncthreads();
            int *t = src;
            src = dst;
            dst = t;
        }
        // the plain indices, in perm (in place when the last round wrote perm:
        // every thread rewrites only its own entries)
        for (int e = threadIdx.x; e < len; e += kLargeBlock) {
            const int v = src[e] & INT_MAX;
            perm[b + e] = v;
            if (inv)
                inv[v] = b + e;
        }
        __syncthreads();
    }
}

// ---- Binning by a stable LSD radix sort (passes of at least kRadixMinN
// particles without an activity mask).  Scattered input gives every block of
// the histogram pass above hundreds of distinct cells, and its global return
// atomics (about one per particle) then bound the binning; a radix sort
// needs none.  Each pass sorts the (cell id, index) pairs stably by the next
// kRadixBits bits of the id: per tile a digit histogram, one scan over the
// digit-major (digit, tile) matrix, then each tile writes its elements to
// their digit's range in index order.  Starting from the indices in order,
// the result is the stable sort by cell, i.e. exactly the permutation of the
// counting sort with per-cell index sorts.
constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixPer = 16;                   // elements per thread and tile
constexpr int kRadixTile = kBlock * kRadixPer;  // 4096 elements per tile
constexpr int64_t kRadixMinN = 1 << 22;         // passes this large bin by radix sort
static_assert(kBlock == kRadixBins, "one thread per digit");

// The lanes of the wavefront whose digit equals this lane's (valid lanes only).
__device__ __forceinline__ unsigned long long digit_peers(unsigned d, bool valid)
{
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const unsigned long long one = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? one : ~one;
    }
    return m;
}

// Cell ids only (the radix path's keys), with the status word.
__global__ __launch_bounds__(kBlock) void k_cellkey(Batch B, unsigned *__restrict__ keys,
                                                    int *__restrict__ status)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < B.ntot)
        keys[i] = (unsigned)particle_cell(B, i, status);
}

// hist[d * ntiles + t] = number of elements of tile t whose digit is d.
__global__ __launch_bounds__(kBlock) void k_radix_hist(const unsigned *__restrict__ keys, int n,
                                                       int shift, int ntiles,
                                                       int *__restrict__ hist)
{
    __shared__ int cnt[kRadixBins];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int base = blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixPer; ++r) {
        const int e = base + r * kBlock + threadIdx.x;
        const bool valid = e < n;
        const unsigned d = valid ? (keys[e] >> shift) & (kRadixBins - 1) : 0u;
        const unsigned long long m = digit_peers(d, valid);
        // the lowest lane of each digit adds its group's count
        if (valid && (m & ((1ull << lane) - 1ull)) == 0ull)
            atomicAdd(&cnt[d], __popcll(m));
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// One pass's scatter, staged through LDS.  Element e of tile t (e = t
// kRadixTile + r kBlock + thread) takes the slot of its digit's range within
// the tile (the exclusive scan of the tile's digit counts) plus the number of
// same-digit elements before it in the tile: those of earlier rounds (run),
// of lower wavefronts in this round (wc) and of lower lanes (a ballot match).
// The tile, so sorted in LDS, is then written out in slot order: each
// digit's elements land as one run at the tile's scanned global offset
// (hist, digit-major: its next entry minus this one is the tile's count).
// vals_in NULL: the values are the indices; inv, when given, receives
// inv[value] = position.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const unsigned *__restrict__ keys_in, const int *__restrict__ vals_in, int n, int shift,
    int ntiles, const int *__restrict__ hist, unsigned *__restrict__ keys_out,
    int *__restrict__ vals_out, int *__restrict__ inv)
{
    __shared__ unsigned lkey[kRadixTile];
    __shared__ int lval[kRadixTile];
    __shared__ int run[kRadixBins];    // next tile slot of each digit
    __shared__ int lbase[kRadixBins];  // first tile slot of each digit
    __shared__ int gbase[kRadixBins];  // first global position of each digit's run
    __shared__ int wc[kBlock / 64][kRadixBins];
    __shared__ int sh[kBlock / 64 + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    {
        const int h = threadIdx.x * ntiles + blockIdx.x;
        const int g = hist[h];
        int total;
        const int ex = block_exclusive_scan(hist[h + 1] - g, sh, &total);
        gbase[threadIdx.x] = g;
        lbase[threadIdx.x] = ex;
        run[threadIdx.x] = ex;
    }
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w)
        wc[w][threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixPer; ++r) {
        const int e = base + r * kBlock + threadIdx.x;
        const bool valid = e < n;
        const unsigned key = valid ? keys_in[e] : 0u;
        const int val = valid ? (vals_in ? vals_in[e] : e) : 0;
        const unsigned d = (key >> shift) & (kRadixBins - 1);
        const unsigned long long m = digit_peers(d, valid);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (valid && below == 0)
            wc[wid][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pos = run[d] + below;
            for (int w = 0; w < wid; ++w)
                pos += wc[w][d];
            lkey[pos] = key;
            lval[pos] = val;
        }
        __syncthreads();
        // digit threadIdx.x: advance its running slot, clear its counts
        int add = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            add += wc[w][threadIdx.x];
            wc[w][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
    const int cnt = n - base < kRadixTile ? n - base : kRadixTile;
    for (int j = threadIdx.x; j < cnt; j += kBlock) {
        const unsigned key = lkey[j];
        const int val = lval[j];
        const unsigned d = (key >> shift) & (kRadixBins - 1);
        const int pos = gbase[d] + (j - lbase[d]);
        keys_out[pos] = key;
        vals_out[pos] = val;
        if (inv)
            inv[val] = pos;
    }
}

// Cell offsets from the sorted ids: offsets[c] = the first slot whose id is
// at least c (n if none), by binary search, one thread per entry c <= ctot.
__global__ __launch_bounds__(kBlock) void k_key_offsets(const unsigned *__restrict__ keys, int n,
                                                        int ctot, int *__restrict__ offsets)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c > ctot)
        return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < (unsigned)c)
            lo = mid + 1;
        else
            hi = mid;
    }
    offsets[c] = lo;
}

// out[k] = in[perm[k]]; an entry outside [0, n) sets the status word and
// writes zero bytes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(const int *__restrict__ perm, int n,
                                                    const T *__restrict__ in, T *__restrict__ out,
                                                    int *__restrict__ status)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n)
        return;
    const unsigned p = (unsigned)perm[k];
    if (p >= (unsigned)n) {
        atomicOr(status, 1);
        out[k] = T{};
        return;
    }
    out[k] = in[p];
}

inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

}  // namespace

int fill_enqueue(sr_ctx *ctx, int *p, int value, int64_t count)
{
    if (count <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(count, kBlock)), dim3(kBlock), 0, ctx->stream, p,
                       value, count);
    return sr_check_launch(ctx, "k_fill");
}

void scan_layout(Bump &b, int m, int **part)
{
    int tiles = (m + kScanTile - 1) / kScanTile;
    *part = b.take<int>(tiles > 0 ? tiles : 1);
}

// out[0..m] = exclusive prefix sums of in[0..m-1], out[m] = total.  `flag`
// is a device int that must be 0 (it is left 0).
int scan_enqueue(sr_ctx *ctx, const int *in, int m, int *part, int *out, int *flag)
{
    if (m <= 0)
        return fill_enqueue(ctx, out, 0, 1);
    int tiles = (m + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_up, dim3(tiles), dim3(kBlock), 0, ctx->stream, in, m, part, tiles,
                       flag);
    hipLaunchKernelGGL(k_scan_down, dim3(tiles), dim3(kBlock), 0, ctx->stream, in, m, part, out);
    return sr_check_launch(ctx, "scan");
}

__global__ void k_clear(ClearList cl)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kClear; ++k)
        if (cl.p[k] && i < cl.n[k])
            cl.p[k][i] = 0;
}

int clear_enqueue(sr_ctx *ctx, const ClearList &cl)
{
    int64_t mx = 0;
    for (int k = 0; k < kClear; ++k)
        if (cl.p[k] && cl.n[k] > mx)
            mx = cl.n[k];
    if (mx <= 0)
        return SR_OK;
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(mx, kBlock)), dim3(kBlock), 0, ctx->stream, cl);
    return sr_check_launch(ctx, "k_clear");
}

void bin_layout(Bump &b, int64_t ntot, int64_t ctot, int nb, BinScratch &s)
{
    size_t nn = (size_t)(ntot > 0 ? ntot : 1);
    s.cid = b.take<int>(nn);
    s.slot = b.take<int>(nn);
    s.count = b.take<int>((size_t)ctot);
    scan_layout(b, (int)ctot, &s.scan_part);
    s.tmp = b.take<int>(nn);
    s.large_list = b.take<int>((size_t)large_class_base((int64_t)nn, kLargeClasses));
    s.large_count = b.take<int>(kLargeClasses + 1);
    s.mass_mixed = b.take<int>((size_t)(nb > 0 ? nb : 1));
    s.scan_flag = b.take<int>(1);
    s.lpt = b.take<int>(64);
    s.n_items = b.take<int>(1);
    s.n_heads = b.take<int>(1);
    s.vtmp = s.ktmp = s.hist = s.hist_part = nullptr;
    if (ntot >= kRadixMinN) {
        const int64_t m = (int64_t)kRadixBins * ((ntot + kRadixTile - 1) / kRadixTile);
        s.vtmp = b.take<int>(nn);
        s.ktmp = b.take<int>(nn);
        s.hist = b.take<int>((size_t)m + 1);
        scan_layout(b, (int)m, &s.hist_part);
    }
}

// The radix path of bin_enqueue (offsets, perm and the inverse).  The ids
// stay in cid in input order, as the counting sort leaves them (the tree
// pass reads them); the passes' keys alternate between tmp and ktmp, their
// indices between vtmp and perm.
static int radix_bin_enqueue(sr_ctx *ctx, const Batch &B, const BinScratch &s, int *offsets,
                             int *perm, int *inv)
{
    const int n = B.ntot;
    const int ntiles = (n + kRadixTile - 1) / kRadixTile;
    const int m = kRadixBins * ntiles;
    unsigned *ids = reinterpret_cast<unsigned *>(s.cid);
    unsigned *kb[2] = {reinterpret_cast<unsigned *>(s.ktmp), reinterpret_cast<unsigned *>(s.tmp)};
    hipLaunchKernelGGL(k_cellkey, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, B,
                       ids, ctx->status);
    int rc = sr_check_launch(ctx, "k_cellkey");
    if (rc)
        return rc;
    const unsigned maxkey = (unsigned)(B.ctot > 1 ? B.ctot - 1 : 1);
    const int bits = 32 - __builtin_clz(maxkey);
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    for (int p = 0; p < passes; ++p) {
        // the last pass writes the indices to perm
        const int *vin = p == 0 ? nullptr : ((passes - p) % 2 == 0 ? perm : s.vtmp);
        int *vout = (passes - p - 1) % 2 == 0 ? perm : s.vtmp;
        // pass p reads the keys pass p - 1 wrote (the ids for p = 0), writes kb[(p + 1) & 1]
        const unsigned *kin = p == 0 ? ids : kb[p & 1];
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kBlock), 0, ctx->stream, kin, n,
                           p * kRadixBits, ntiles, s.hist);
        if ((rc = sr_check_launch(ctx, "k_radix_hist")) ||
            (rc = scan_enqueue(ctx, s.hist, m, s.hist_part, s.hist, s.scan_flag)))
            return rc;
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kBlock), 0, ctx->stream, kin,
                           vin, n, p * kRadixBits, ntiles, s.hist, kb[(p + 1) & 1], vout,
                           p == passes - 1 ? inv : nullptr);
        if ((rc = sr_check_launch(ctx, "k_radix_scatter")))
            return rc;
    }
    hipLaunchKernelGGL(k_key_offsets, dim3(blocks_for((int64_t)B.ctot + 1, kBlock)), dim3(kBlock),
                       0, ctx->stream, kb[passes & 1], n, B.ctot, offsets);
    return sr_check_launch(ctx, "k_key_offsets");
}

// Enqueue the whole binning pass.  sorted and chunk_count may be NULL (then
// no gather and no item counts); tcount (per-cell active counts) is given
// exactly when the pass carries an activity mask.
int bin_enqueue(sr_ctx *ctx, const Batch &B, const BinScratch &s, int *offsets, int *perm,
                float4 *sorted, int *chunk_count, int *tcount)
{
    int rc;
    {
        ClearList cl{};
        cl.p[0] = s.count;
        cl.n[0] = B.ctot;
        cl.p[1] = s.large_count;
        cl.n[1] = kLargeClasses + 1;
        cl.p[2] = s.mass_mixed;
        cl.n[2] = B.nb;
        cl.p[3] = s.scan_flag;
        cl.n[3] = 1;
        cl.p[4] = s.lpt;
        cl.n[4] = 64;
        cl.p[5] = s.n_items;
        cl.n[5] = 1;
        cl.p[6] = s.n_heads;
        cl.n[6] = 1;
        if ((rc = clear_enqueue(ctx, cl)))
            return rc;
    }
    const int n = B.ntot;
    // only single-box passes carry an activity mask (the batched forms pass
    // none); its cell flags go to chunk_count and its active counts to
    // tcount, which k_segsort then turns into item counts
    const bool masked = !B.boxes && B.one.active != nullptr;
    if (masked && !(chunk_count && tcount))
        return sr_fail(ctx, SR_EINVAL, "an activity mask needs item and target counts");
    if (masked && ((rc = fill_enqueue(ctx, chunk_count, 0, B.ctot)) ||
                   (rc = fill_enqueue(ctx, tcount, 0, B.ctot))))
        return rc;
    // the arrival ranks are not needed once the cells are sorted: their
    // buffer takes the inverse permutation
    int *inv = sorted ? s.slot : nullptr;
    if (!masked && s.vtmp && n >= kRadixMinN) {
        if ((rc = radix_bin_enqueue(ctx, B, s, offsets, perm, inv)))
            return rc;
        if (sorted) {
            hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0,
                               ctx->stream, B, inv, sorted, s.mass_mixed, nullptr, nullptr);
            if ((rc = sr_check_launch(ctx, "k_gather")))
                return rc;
        }
        return SR_OK;
    }
    if (n > 0) {
        if (masked)
            hipLaunchKernelGGL(k_cellid<true>, dim3(blocks_for(n, kCellidBlock)), dim3(kBlock), 0,
                               ctx->stream, B, s.cid, s.slot, s.count, ctx->status, chunk_count,
                               tcount);
        else
            hipLaunchKernelGGL(k_cellid<false>, dim3(blocks_for(n, kCellidBlock)), dim3(kBlock),
                               0, ctx->stream, B, s.cid, s.slot, s.count, ctx->status, nullptr,
                               nullptr);
        if ((rc = sr_check_launch(ctx, "k_cellid")))
            return rc;
        if (masked) {
            hipLaunchKernelGGL(k_relevant, dim3(blocks_for(B.ctot, kBlock)), dim3(kBlock), 0,
                               ctx->stream, B.one.g, chunk_count, s.count);
            if ((rc = sr_check_launch(ctx, "k_relevant")))
                return rc;
        }
    }
    if ((rc = scan_enqueue(ctx, s.count, B.ctot, s.scan_part, offsets, s.scan_flag)))
        return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, ctx->stream,
                           s.cid, s.slot, n, offsets, masked ? B.one.active : nullptr, perm);
        if ((rc = sr_check_launch(ctx, "k_scatter")))
            return rc;
    }
    hipLaunchKernelGGL(k_segsort, dim3(blocks_for(B.ctot, kBlock / 64 * kSegGroup)), dim3(kBlock), 0,
                       ctx->stream, B, offsets, perm, s.large_list, s.large_count, inv,
                       masked ? chunk_count : nullptr, masked ? tcount : nullptr);
    if ((rc = sr_check_launch(ctx, "k_segsort")))
        return rc;
    if (n > kLargeCell) {
        // one block per CU, each with the whole LDS (kLdsCell indices)
        static const hipError_t lds_ok = hipFuncSetAttribute(
            (const void *)k_segsort_large, hipFuncAttributeMaxDynamicSharedMemorySize,
            kLdsCell * (int)sizeof(int));
        if (lds_ok != hipSuccess)
            return sr_fail(ctx, SR_EDEVICE, "k_segsort_large: %d bytes of LDS not available",
                           kLdsCell * (int)sizeof(int));
        int max_large = n / (kLargeCell + 1) + 1;
        int grid = max_large < 256 ? max_large : 256;
        hipLaunchKernelGGL(k_segsort_large, dim3(grid), dim3(kLargeBlock),
                           kLdsCell * sizeof(int), ctx->stream, B, offsets, perm, s.tmp,
                           s.large_list, s.large_count, inv);
        if ((rc = sr_check_launch(ctx, "k_segsort_large")))
            return rc;
    }
    if (sorted && n > 0) {
        hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, ctx->stream,
                           B, inv, sorted, s.mass_mixed, masked ? s.cid : nullptr,
                           masked ? offsets : nullptr);
        if ((rc = sr_check_launch(ctx, "k_gather")))
            return rc;
    }
    return SR_OK;
}

extern "C" int sr_bin(sr_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                      const sr_box *box, double cell, int32_t *cell_offsets, int32_t *perm)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n=%lld out of range", (long long)n);
    if (!cell_offsets || (n > 0 && (!x || !y || !z || !perm)))
        return sr_fail(ctx, SR_EINVAL, "NULL pointer");
    Batch B{};
    int rc = sr_make_geom(ctx, box, cell, &B.one.g);
    if (rc)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    B.nb = 1;
    B.ntot = (int)n;
    B.ctot = B.one.g.ncell;
    B.one.n = (int)n;
    B.one.x = x;
    B.one.y = y;
    B.one.z = z;
    Bump sz{nullptr, 0, 0};
    BinScratch s;
    bin_layout(sz, n, B.ctot, 1, s);
    if ((rc = sr_arena_reserve(ctx, sz.off)))
        return rc;
    Bump b{ctx->arena, 0, ctx->arena_cap};
    bin_layout(b, n, B.ctot, 1, s);
    return bin_enqueue(ctx, B, s, cell_offsets, perm, nullptr, nullptr, nullptr);
}

extern "C" int sr_permute(sr_ctx *ctx, const int32_t *perm, int64_t n, int32_t elem_bytes,
                          const void *in, void *out)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n=%lld out of range", (long long)n);
    if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16)
        return sr_fail(ctx, SR_EINVAL, "elem_bytes must be 4, 8 or 16 (got %d)", elem_bytes);
    if (n == 0)
        return SR_OK;
    if (!perm || !in || !out)
        return sr_fail(ctx, SR_EINVAL, "NULL pointer");
    if (in == out)
        return sr_fail(ctx, SR_EINVAL, "in and out must be different arrays");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    const int ni = (int)n;
    const dim3 grid(blocks_for(n, kBlock)), block(kBlock);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_permute<unsigned>, grid, block, 0, ctx->stream, perm, ni,
                           static_cast<const unsigned *>(in), static_cast<unsigned *>(out),
                           ctx->status);
    else if (elem_bytes == 8)
        hipLaunchKernelGGL(k_permute<unsigned long long>, grid, block, 0, ctx->stream, perm, ni,
                           static_cast<const unsigned long long *>(in),
                           static_cast<unsigned long long *>(out), ctx->status);
    else
        hipLaunchKernelGGL(k_permute<uint4>, grid, block, 0, ctx->stream, perm, ni,
                           static_cast<const uint4 *>(in), static_cast<uint4 *>(out),
                           ctx->status);
    return sr_check_launch(ctx, "k_permute");
}
