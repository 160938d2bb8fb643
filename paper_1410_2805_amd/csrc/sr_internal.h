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
    int *status = nullptr;      // device status word (bit 0: bad coordinate)
    int64_t *stats = nullptr;   // device counters for sr_pair_stats
    std::string err;
    int xsplit = 2;             // sub-cells per chaining cell along x in sr_force
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
struct Geom {
    double len[3];
    double inv[3];
    float lenf[3];
    int nc[3];
    int ncell;
    int periodic;
    int hx;
    double skin;
};

constexpr int kMaxXsplit = 4;

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
    int *cid;         // [n] cell id of each original particle
    int *slot;        // [n] arrival rank within its cell (atomic, unordered)
    int *count;       // [ncell] particles per cell
    int *scan_part;   // [scan tiles] partial sums
    int *tmp;         // [n] ping-pong buffer of the large-cell merge
    int *large_list;  // [max_large] cells too big for one wavefront's LDS
    int *large_count; // [1]
    int *mass_mixed;  // [1] set to 1 by the gather if any mass differs from m[0]
};

// Host helpers (sr_ctx.cpp)
int sr_fail(sr_ctx *ctx, int code, const char *fmt, ...);
int sr_make_geom(sr_ctx *ctx, const sr_box *box, double cell, Geom *g, int xsplit = 1);
int sr_arena_reserve(sr_ctx *ctx, size_t need);
int sr_check_launch(sr_ctx *ctx, const char *what);
// When timing is on: index of a fresh 3-event record, else -1.
int sr_timing_begin(sr_ctx *ctx);
void sr_timing_mark(sr_ctx *ctx, int rec, int which);

// Binning (sr_bin.hip)
void bin_layout(Bump &b, int64_t n, const Geom &g, BinScratch &s);
int bin_enqueue(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *m,
                int n, const Geom &g, const BinScratch &s, int *offsets, int *perm,
                float4 *sorted, int *chunk_count);
void scan_layout(Bump &b, int m, int **part);
int scan_enqueue(sr_ctx *ctx, const int *in, int m, int *part, int *out);
int fill_enqueue(sr_ctx *ctx, int *p, int value, int64_t count);

constexpr int kLargeCell = 1024;   // cells above this are sorted by a whole block
constexpr int kChunk = 64;         // maximum targets per force work item
constexpr int kMaxSplit = 16;      // at most 16 lane groups share one target

// A force work item with nt targets gives each target S = floor(64/nt)
// lanes (capped), which take disjoint slices of every source tile.
__host__ __device__ inline int split_for(int nt)
{
    int s = nt > 0 ? 64 / nt : kMaxSplit;
    return s < 1 ? 1 : (s > kMaxSplit ? kMaxSplit : s);
}

// Number of work items a cell of n targets is cut into: the cheapest
// candidate count under a cost model in which an item costs 1/S of a
// full-wavefront pass over its sources plus 5 % fixed overhead.  Chunk k of
// q covers targets [k n / q, (k + 1) n / q).
__host__ __device__ inline int chunks_for(int n)
{
    if (n <= 0)
        return 0;
    const int q0 = (n + kChunk - 1) / kChunk;
    // chunks below 16 targets never pay off (S is capped); this also bounds
    // the item count by (non-empty cells) + n / 16
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
