// Internal declarations shared by the translation units of libsr.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "sr.h"

struct sr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char *arena = nullptr;      // one device allocation for all scratch
    size_t arena_cap = 0;
    size_t high_water = 0;
    bool fixed = false;         // fixed-size arena: never regrow
    hipEvent_t handoff = nullptr;  // orders a new stream after the old one (sr_set_stream)
    int *status = nullptr;      // device status word (bit 0: bad coordinate)
    int64_t *stats = nullptr;   // device counters for sr_pair_stats
    std::string err;
    int xsplit = 1;             // sub-cells per chaining cell along x in sr_force
    int order = 1;              // work-item order: 0 cell order, 1 cost buckets (LPT)
    int persistent = 0;         // 1: persistent workgroups pull items from a counter
    bool timing = false;        // record events around sr_force phases
    std::vector<hipEvent_t> events;  // 3 per recorded call
    size_t events_used = 0;
};

// Chaining-mesh geometry as the kernels see it.  inv = dims / len is formed
// on the host in FP64 and the cell of a coordinate is floor(x * inv) in FP64.
//
// For the pair loop the x axis may be cut finer than the chaining cell:
// hx = xsplit sub-cells per chaining cell along x, so the stencil is
// (2 hx + 1) x 3 x 3 cells.  Rows along x stay contiguous in the sorted
// order, and the searched x extent shrinks from 3 to 2 + 1/hx chaining
// cells (fewer candidate pairs for the same cutoff).
//
// Split coordinates (split != 0, periodic boxes only): a particle is given
// as its chaining cell (cx, cy, cz), packed 10 bits each into cell3, and a
// float32 offset from that cell's lower corner.  The pair loop then works
// entirely in cell-relative float32 coordinates (w = cell widths, FP64).
struct Geom {
    double len[3];
    double inv[3];
    double w[3];
    float lenf[3];
    int nc[3];
    int ncell;
    int periodic;
    int hx;
    int split;
    double skin;
    // cell / (nc[0] nc[1]) and rem / nc[0] by multiply and shift (div_const)
    unsigned div_m[2];
    int div_s[2];
};

// Constants for the exact quotient n / d of any 0 <= n < 2^31 by a fixed
// d >= 1 (Granlund and Montgomery's method): with s = ceil(log2 d) and
// m = floor(2^(31+s) / d) + 1 < 2^32, n m / 2^(31+s) exceeds n / d by less
// than n / 2^(31+s) < 2^-s <= 1 / d, so its floor is floor(n / d).
inline void div_const(unsigned d, unsigned *m, int *s)
{
    int l = 0;
    while ((1ull << l) < d)
        ++l;
    *s = l;
    *m = (unsigned)(((1ull << (31 + l)) / d) + 1ull);
}

__host__ __device__ inline int div_by(int n, unsigned m, int s)
{
    return (int)(((unsigned long long)(unsigned)n * m) >> (31 + s));
}

constexpr int kSplitMaxCells = 1023;  // per axis, split coordinates

constexpr int kMaxXsplit = 4;
constexpr double kMaxSide = 131072.0;  // largest box side (padding lies far beyond)

// One box of a batch.  Particles of all boxes are numbered consecutively
// (box b owns [pbase, pbase + n)) and so are their cells ([cbase, cbase +
// g.ncell)); inputs and outputs stay in the caller's per-box arrays.
struct BoxDesc {
    Geom g;
    int pbase, n, cbase, _pad;
    const float *x, *y, *z, *m;   // positions, or cell offsets when g.split
    const int *cell3;             // split coordinates: packed chaining cells
    // optional, single-box passes: 0 inactive, 1 active, 2 active and its
    // cell cut into finer items; only active particles are targets (every
    // particle stays a source) and only their accelerations are written
    const unsigned char *active;
    float *ax, *ay, *az;
};

// A batch as the kernels see it (passed by value).  A single box travels
// inside the kernel arguments (`one`); larger batches read a device table.
struct Batch {
    const BoxDesc *boxes;  // device table, or nullptr when nb == 1
    const int *pstart;     // [nb + 1] first particle of each box
    const int *cstart;     // [nb + 1] first cell of each box
    int nb;
    int ntot;
    int ctot;
    int _pad;
    BoxDesc one;
};

// Largest b with start[b] <= v (boxes with no particles are skipped).
__device__ __forceinline__ int find_box(const int *start, int nb, int v)
{
    if (nb == 1)
        return 0;
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ const BoxDesc &box_at(const Batch &B, int b)
{
    return B.boxes ? B.boxes[b] : B.one;
}

// LDS hash table of a block's distinct cell ids: kHash slots for at most
// 1024 keys, so the linear probe always ends.  Returns the slot of `id`,
// inserting it when absent (hkey slots start at -1).
constexpr int kHash = 2048;
__device__ __forceinline__ int lds_hash_slot(int *hkey, int id)
{
    int h = (int)(((unsigned)id * 2654435761u) >> 21) & (kHash - 1);
    for (;;) {
        const int old = atomicCAS(&hkey[h], -1, id);
        if (old == -1 || old == id)
            return h;
        h = (h + 1) & (kHash - 1);
    }
}

// Scalars of the pair loop in the form the kernel evaluates.
//   se = s + eps is formed directly by the FMA chain, the cutoff test is
//   se < rcut with rcut = fl32(r_max^2 + eps), and the polynomial is
//   re-expanded around -eps so that p(s) = q(se):  q_k = sum_{j>=k}
//   C(j,k) c_j (-eps)^(j-k), formed in FP64 and rounded once to float32.
//   nq holds -q_1..-q_5 (negated for the fused subtraction) and q0 = q_0.
struct ForceParams {
    float eps;
    float rcut;
    float q0;
    float nq[6];  // nq[1..5] used
};

// Bump allocator over the context arena for one call.
struct Bump {
    char *base;
    size_t off;
    size_t cap;
    template <class T>
    T *take(size_t count) {
        size_t a = (off + 255) & ~size_t(255);
        off = a + count * sizeof(T);
        return base ? reinterpret_cast<T *>(base + a) : nullptr;
    }
};

// Scratch of one binning pass (sorted-slot order), carved from the arena.
struct BinScratch {
    int *cid;         // [ntot] global cell id of each particle
    int *slot;        // [ntot] arrival rank within its cell (atomic, unordered)
    int *count;       // [ctot] particles per cell
    int *scan_part;   // [scan tiles] partial sums
    int *tmp;         // [ntot] ping-pong buffer of the large-cell merge
    int *large_list;  // cells too big for one wavefront's LDS, by size class
    int *large_count; // [9] large cells per size class, then the block sort's work counter
    int *mass_mixed;  // [nb] box b: 1 if any of its masses differs from its first
    int *scan_flag;   // [1] last-block counter of the scans (kept at 0)
    int *lpt;         // [64] key totals and cursors of the longest-first item order
    int *n_items;     // [1] force work items appended by k_items
    int *n_heads;     // [1] chunks cut into sub-items, appended by k_items
    // radix-sort binning (passes of many particles; null otherwise)
    int *vtmp;        // [ntot] index ping-pong buffer
    int *ktmp;        // [ntot] key ping-pong buffer (with tmp; cid keeps the ids)
    int *hist;        // [digits * tiles + 1] per-tile digit counts, scanned in place
    int *hist_part;   // scan partials of hist
};

// Up to seven int buffers zeroed by one kernel launch.
constexpr int kClear = 7;
struct ClearList {
    int *p[kClear];
    int64_t n[kClear];
};

// Everything a force pass needs beyond binning.
struct ForceScratch {
    BinScratch bin;
    int *offsets;     // [ctot + 1]
    int *perm;        // [ntot]
    float4 *sorted;   // [ntot] (x, y, z, m) in cell order
    int *chunk_count; // [ctot] masked passes: activity flags, then chunks per cell
    int4 *items;      // [item bound] in cell order
    int *item_cost;   // [item bound] cost bucket of each item
    int4 *items_lpt;  // [item bound] items by decreasing cost bucket
    int *queue;       // [1] persistent work counter
    double *mom_part; // [nb * kRedBlocks * 3]
    float4 *part;     // [(kMaxSrcSplit - 1) * ntot] partial sums of sub-items 1.., or null
    int4 *heads;      // [chunk bound] first sub-items of the chunks cut into sub-items
    int *tcount;      // [ctot] active targets per cell (masked passes), or null
};

constexpr int kRedBlocks = 512;    // FP64 reduction blocks per box (at most)
constexpr int kLargeCell = 1024;   // cells above this are sorted by a whole block
constexpr int kChunk = 64;         // maximum targets per work item at one target per lane
constexpr int kChunk2 = 128;       // ... and at two targets per lane (chaining-mesh pass)
constexpr int kMaxSplit = 16;      // at most 16 lane groups share one target
constexpr int kLptBlock = 1024;    // items per block of the cost-bucket sort

// Looks up the device address of sr_force_static's fixed scratch array on
// `device` (current) once (sr_noalloc.hip).
int static_scratch_setup(int device);

// Host helpers (sr_ctx.cpp)
int sr_fail(sr_ctx *ctx, int code, const char *fmt, ...);
int sr_make_geom(sr_ctx *ctx, const sr_box *box, double cell, Geom *g, int xsplit = 1);
int sr_arena_reserve(sr_ctx *ctx, size_t need);
int sr_check_launch(sr_ctx *ctx, const char *what);
// When timing is on: index of a fresh 3-event record, else -1.
int sr_timing_begin(sr_ctx *ctx);
void sr_timing_mark(sr_ctx *ctx, int rec, int which);

// Binning (sr_bin.hip)
void bin_layout(Bump &b, int64_t ntot, int64_t ctot, int nb, BinScratch &s);
int bin_enqueue(sr_ctx *ctx, const Batch &B, const BinScratch &s, int *offsets, int *perm,
                float4 *sorted, int *chunk_count, int *tcount);
void scan_layout(Bump &b, int m, int **part);
int scan_enqueue(sr_ctx *ctx, const int *in, int m, int *part, int *out, int *flag);
int fill_enqueue(sr_ctx *ctx, int *p, int value, int64_t count);
int clear_enqueue(sr_ctx *ctx, const ClearList &cl);

// Force pass (sr_force.hip)
// Items of a pass at most; masked: a pass with an activity mask, whose
// flagged cells may take finer items and sub-items.
int64_t item_bound(int64_t ntot, int64_t ctot, bool split = false);
// masked: a pass with an activity mask (its flagged cells are cut into
// sub-items); split_ok: some box of the pass may cut its chunks
// (box_splits).  Either gives the pass sub-item storage.
void force_layout(Bump &b, int64_t ntot, int64_t ctot, int nb, ForceScratch &s, bool masked,
                  bool split_ok);
int check_box_args(sr_ctx *ctx, const sr_box *box, double cell, float r_max, int xsplit,
                   Geom *g);
int check_force_params(sr_ctx *ctx, float r_max, float eps, const float *poly);
ForceParams make_params(float r_max, float eps, const float *poly);
// Longest-first order (counting sort on 5-bit cost buckets) of the *n_items
// items; bound >= the item count; lpt: int[64], zero on entry (BinScratch).
int lpt_sort_enqueue(sr_ctx *ctx, const int4 *items, const int *item_cost, const int *n_items,
                     int64_t bound, int *lpt, int4 *out);
int single_batch(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *mass,
                 int64_t n, const sr_box *box, double cell, float r_max, int xsplit, float *ax,
                 float *ay, float *az, Batch *B);
int momentum_enqueue(sr_ctx *ctx, const Batch &B, double *part, double *mom);
int force_split_masked(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                       const float *oz, const float *mass, int64_t n, const sr_box *box,
                       double cell, float r_max, float eps, const float poly[6], float *ax,
                       float *ay, float *az, double *momentum3, const unsigned char *active,
                       size_t *bytes);
// Enqueue bin + items (+ cost order) + pair loop + momentum for a batch.
// order: 0 cell order, 1 cost buckets; persistent: one wave per CU slot
// pulling items from a counter.  mom: device double[3 * nb] or nullptr.
int force_enqueue(sr_ctx *ctx, const Batch &B, const ForceScratch &s, const ForceParams &fp,
                  int order, int persistent, double *mom, int timing_rec);

// A force work item with nt targets gives each target S = floor(64/nt)
// lanes (capped), which take disjoint slices of every source tile.
__host__ __device__ constexpr inline int split_for(int nt)
{
    int s = nt > 0 ? 64 / nt : kMaxSplit;
    return s < 1 ? 1 : (s > kMaxSplit ? kMaxSplit : s);
}

// Number of work items a cell of n targets is cut into.  Up to 256 targets
// the cheapest candidate count under a cost model in which an item costs
// 1/S of a full-wavefront pass over its sources plus 5 % fixed overhead;
// beyond, chunks of at most 64 (S = 1 is then efficient).  Chunk k of q
// covers targets [k n / q, (k + 1) n / q).  The count never exceeds
// max(ceil(n / 64), n / 16), which bounds the items by (non-empty cells) +
// n / 16.
__host__ __device__ constexpr inline int chunks_for(int n)
{
    if (n <= 0)
        return 0;
    const int q0 = (n + kChunk - 1) / kChunk;
    if (n > 4 * kChunk)
        return q0;
    const int qmax = q0 > n / 16 ? q0 : n / 16;
    float best = 3.0e38f;
    int bq = q0;
    for (int q = q0; q <= qmax; ++q) {
        float c = 0.05f * (float)q;
        for (int k = 0; k < q; ++k) {
            int sz = (k + 1) * n / q - k * n / q;
            c += 1.0f / (float)split_for(sz);
        }
        if (c < best) {
            best = c;
            bq = q;
        }
    }
    return bq;
}

// Cost of one wavefront pass over a source at two targets per lane (two pair
// evaluations per lane) relative to one target per lane: the ratio of the
// instruction counts of the two pair loops per source (both loops issue the
// same instructions per pair).
constexpr float kTwoPerLane = 2.0f;

// Shape of a chaining-mesh work item of nt targets (nt <= kChunk2): tpl
// targets per lane (1, or 2 with lane t holding targets t and t + ceil(nt/2))
// and S lane groups, whichever needs fewer issue slots per source; returns
// that cost in full-wavefront passes per source.
__host__ __device__ constexpr inline float item_shape(int nt, int *tpl, int *S)
{
    const float c1 = nt <= kChunk ? 1.0f / (float)split_for(nt) : 3.0e38f;
    const int s2 = split_for((nt + 1) / 2);
    const float c2 = kTwoPerLane / (float)s2;
    if (c1 <= c2) {
        *tpl = 1;
        *S = split_for(nt);
        return c1;
    }
    *tpl = 2;
    *S = s2;
    return c2;
}

// chunks_for for the chaining-mesh pass, whose items may take two targets per
// lane: up to 256 targets the cheapest count of equal chunks under the same
// model with item_shape's cost; beyond, full chunks of kChunk2 and the last
// kChunk2 + 1 .. 2 kChunk2 targets cut as that model cuts them (mesh_chunks).
// The count never exceeds max(ceil(n / 64), n / 16) either.
__host__ __device__ constexpr inline int mesh_chunks_for(int n)
{
    if (n <= 0)
        return 0;
    if (n > 4 * kChunk) {
        const int full = (n - kChunk2 - 1) / kChunk2;
        return full + mesh_chunks_for(n - full * kChunk2);
    }
    const int q0 = (n + kChunk2 - 1) / kChunk2;
    const int qmax = q0 > n / 16 ? q0 : n / 16;
    float best = 3.0e38f;
    int bq = q0;
    for (int q = q0; q <= qmax; ++q) {
        float c = 0.05f * (float)q;
        for (int k = 0; k < q; ++k) {
            int tpl = 0, S = 0;
            c += item_shape((k + 1) * n / q - k * n / q, &tpl, &S);
        }
        if (c < best) {
            best = c;
            bq = q;
        }
    }
    return bq;
}

// chunks_for and mesh_chunks_for of every n <= 4 kChunk, evaluated at compile
// time: the device takes one lookup instead of the cost model's loops.
struct ChunkTables {
    unsigned char tree[4 * kChunk + 1];
    unsigned char mesh[4 * kChunk + 1];
};

constexpr ChunkTables make_chunk_tables()
{
    ChunkTables t{};
    for (int n = 0; n <= 4 * kChunk; ++n) {
        t.tree[n] = (unsigned char)chunks_for(n);
        t.mesh[n] = (unsigned char)mesh_chunks_for(n);
    }
    return t;
}

namespace {
__constant__ const ChunkTables kChunkTab = make_chunk_tables();
}  // namespace

__device__ __forceinline__ int tree_chunks(int n)
{
    return n <= 4 * kChunk ? (n > 0 ? kChunkTab.tree[n] : 0) : (n + kChunk - 1) / kChunk;
}

// Beyond 4 kChunk targets: full chunks of kChunk2, then the remaining
// kChunk2 + 1 .. 2 kChunk2 targets cut as the small-cell table cuts them.
// Against ceil(n / kChunk2) equal chunks this leaves fewer lanes idle: a
// full chunk fills all 64 lanes at two targets per lane, and only the
// remainder's chunks may not (a CPU model of the item shapes puts the idle
// share of the pair loop's issue slots on nfw256 at 0.6 % against 2.6 %).
__device__ __forceinline__ int mesh_full_chunks(int n)
{
    return n > 4 * kChunk ? (n - kChunk2 - 1) / kChunk2 : 0;
}

__device__ __forceinline__ int mesh_chunks(int n)
{
    if (n <= 4 * kChunk)
        return n > 0 ? kChunkTab.mesh[n] : 0;
    const int full = mesh_full_chunks(n);
    return full + kChunkTab.mesh[n - full * kChunk2];
}

// Targets [*lo, *hi) of chunk k of q of a cell of len targets: with mesh,
// the layout of mesh_chunks (q its count), else q nearly equal parts [k len /
// q, (k + 1) len / q).
__device__ __forceinline__ void chunk_range(int len, int q, int k, bool mesh, int *lo, int *hi)
{
    int base = 0;
    if (mesh && len > 4 * kChunk) {
        const int full = mesh_full_chunks(len);
        if (k < full) {
            *lo = k * kChunk2;
            *hi = *lo + kChunk2;
            return;
        }
        base = full * kChunk2;
        len -= base;
        q -= full;
        k -= full;
    }
    // k len fits in 32 bits below 46341 targets (q <= len)
    const bool small = len <= 46340;
    *lo = base + (small ? k * len / q : (int)((long long)k * len / q));
    *hi = base + (small ? (k + 1) * len / q : (int)((long long)(k + 1) * len / q));
}

// Work items.  A cell's targets are cut into q chunks (chunk_range); a chunk
// is one item, or ns sub-items that take
// consecutive parts [sk T / ns, (sk + 1) T / ns) of the T stencil sources,
// so that the pairs of a dense cell spread over more wavefronts and no
// single wavefront holds up the end of the pass (a chunk of P target-source
// pairs takes ceil(P / kSplitPairs) sub-items, at most kMaxSrcSplit).  Cells
// flagged for finer items (multilevel passes) are cut so in any box, and
// their short chunks into chunks of at most kFineChunk targets instead.  A
// sub-item leaves partial sums, which a second pass adds in sub-item order.
constexpr int kMaxSrcSplit = 8;       // sub-items per chunk at most
constexpr int kFineChunk = 32;        // targets per item of short chunks in flagged cells
constexpr int kFineSources = 4096;    // stencil sources per sub-item of those chunks, about
constexpr long long kSplitPairs = 1 << 20;  // target-source pairs per sub-item, about
constexpr int64_t kSplitMaxN = 1 << 22;     // boxes of at most this many particles cut other chunks

// Whether the chunks of a box of n particles (other than those of cells
// flagged for finer items) may be cut into sub-items: a property of the box
// alone, so that a box gives the same sums alone and in a batch.  Larger
// boxes have enough items to keep every wavefront busy to the end.
__host__ __device__ inline bool box_splits(int64_t n)
{
    return n <= kSplitMaxN;
}
constexpr int kFineFlag = 1 << 30;    // chunk_count bit: cell flagged for finer items
constexpr int kMaxBatchBoxes = 1 << 17;

// Item layout: {cell (global), first sorted slot, targets, S | (tpl - 1) << 5
// | sk << 6 | (ns - 1) << 10 | box << 14}.
__host__ __device__ inline int item_word(int S, int tpl, int sk, int ns, int box)
{
    return S | (tpl - 1) << 5 | sk << 6 | (ns - 1) << 10 | box << 14;
}

// Stencil size of cell c (global id): the sources of its 9 x-rows of 2 hx + 1
// cells (shifts aside); also its box, first sorted slot and particle count.
__device__ inline long long cell_stencil(const Batch &B, const int *__restrict__ offsets, int c,
                                         int *box_out, int *b_out, int *len_out)
{
    const int box = find_box(B.cstart, B.nb, c);
    const BoxDesc &d = box_at(B, box);
    const Geom &g = d.g;
    const int b = offsets[c];
    const int len = offsets[c + 1] - b;
    const int lc = c - d.cbase, plane = g.nc[0] * g.nc[1];
    const int cz = lc / plane, cy = (lc - cz * plane) / g.nc[0];
    const int cx = lc - cz * plane - cy * g.nc[0];
    const int *off = offsets + d.cbase;
    long long src = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        int ny = cy + r % 3 - 1, nz = cz + r / 3 - 1;
        if (g.periodic) {
            ny = ny < 0 ? ny + g.nc[1] : (ny >= g.nc[1] ? ny - g.nc[1] : ny);
            nz = nz < 0 ? nz + g.nc[2] : (nz >= g.nc[2] ? nz - g.nc[2] : nz);
        } else if (ny < 0 || ny >= g.nc[1] || nz < 0 || nz >= g.nc[2]) {
            continue;
        }
        const int row = g.nc[0] * (ny + g.nc[1] * nz);
        const int lo = cx - g.hx, hi = cx + g.hx, n0 = g.nc[0];
        if (g.periodic) {
            if (lo < 0)
                src += (off[row + hi + 1] - off[row]) + (off[row + n0] - off[row + lo + n0]);
            else if (hi >= n0)
                src += (off[row + n0] - off[row + lo]) + (off[row + hi - n0 + 1] - off[row]);
            else
                src += off[row + hi + 1] - off[row + lo];
        } else {
            const int a = lo > 0 ? lo : 0, e = hi < n0 - 1 ? hi : n0 - 1;
            src += off[row + e + 1] - off[row + a];
        }
    }
    *box_out = box;
    *b_out = b;
    *len_out = len;
    return src;
}

// Sub-item sk of chunk k of a cell (first sorted slot b, len targets, q
// chunks laid out as mesh_chunks lays them out (mesh) or equal, ns sub-items
// per chunk, src stencil sources), shaped by item_shape;
// *bucket is floor(log2(cost)), cost = (the sub-item's sources) x (the
// shape's cost per source) + 64 (wavefront iterations plus overhead).
__device__ inline int4 cell_item(int c, int box, int b, int len, int q, bool mesh, int k, int ns,
                                 int sk, long long src, int *bucket)
{
    int lo, hi;
    chunk_range(len, q, k, mesh, &lo, &hi);
    int tpl, S;
    const float pass = item_shape(hi - lo, &tpl, &S);
    const long long cost = (long long)((float)(src / ns) * pass) + 64;
    *bucket = 63 - __clzll((unsigned long long)cost);
    return make_int4(c, b + lo, hi - lo, item_word(S, tpl, sk, ns, box));
}
