/*
 * sr.h -- C ABI of libsr, the MI355X (gfx950) short-range particle-particle
 * force of the HACC hybrid N-body method (Habib et al., "HACC: Simulating Sky
 * Surveys on State-of-the-Art Supercomputing Architectures", arXiv:1410.2805).
 *
 * What is computed
 *   For every target particle i that is not passive,
 *
 *     a_i = sum_{j != i, s_ij < r_max^2}  m_j f_SR(s_ij) d_ij,
 *     f_SR(s) = (s + eps)^(-3/2) - p(s),   p(s) = sum_{k=0..5} c_k s^k,
 *
 *   d_ij = x_j - x_i (minimum image in a periodic box), s_ij = d_ij . d_ij:
 *   Eq. (force) of Sec. 3.1, with p the fifth-order polynomial that stands
 *   in for the filtered grid force of Sec. 2.4 (Eq. (fitform)), eps the
 *   Plummer softening added to s, G = 1 and lengths in grid units (Sec. 2.6).
 *   Pairs are found through a chaining mesh of cells at least as wide as the
 *   cutoff, searched over each cell and its 26 neighbours (Sec. 2.4, last
 *   paragraph; Sec. 3.1, fixed bins of the short-range scale).  Passive
 *   particles of a non-periodic (overloaded) domain -- those closer than the
 *   skin width to a face -- receive no short-range force but act as sources
 *   (Sec. 2.2).
 *
 * Conventions (all entry points)
 *   - Particle data are float32 structure-of-arrays in DEVICE memory owned by
 *     the caller: x[n], y[n], z[n], mass[n]; outputs likewise.  The library
 *     never frees caller memory.  Coordinates must satisfy 0 <= x < L.
 *   - Scratch memory comes from the context's arena (a single device
 *     allocation, reused by every call; see sr_ctx_create).
 *   - Every call only enqueues work on the context's HIP stream and returns;
 *     it never waits for the device.  sr_sync waits and reports errors that
 *     the device detected (SR_ERANGE for a coordinate outside [0, L) or NaN).
 *   - Argument errors are reported synchronously by a negative return value;
 *     sr_last_error gives a message.  Nothing is enqueued in that case.
 *   - Output sizes are fixed by (box, cell, n) and can be computed on the host
 *     with sr_grid_dims.
 *   - A context is used by one host thread at a time.
 */
#ifndef SR_H
#define SR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SR_OK = 0,
    SR_EDEVICE = -5,  /* HIP runtime error */
    SR_ENOMEM = -12,  /* scratch arena too small (fixed-size arena) or allocation failed */
    SR_EBUSY = -16,   /* serving: no free slot / HBM budget exhausted */
    SR_EINVAL = -22,  /* invalid argument */
    SR_ERANGE = -34   /* device-detected: coordinate outside [0, L) or NaN */
};

/* Box [0, len[0]) x [0, len[1]) x [0, len[2]), each side at most 131072
 * (SR_EINVAL beyond) and exactly representable in float32.
 *   periodic != 0 : periodic in all three axes, minimum-image separations.
 *   periodic == 0 : open domain of an overloaded node (Sec. 2.2); particles
 *                   whose distance to the nearest face is < skin (strictly,
 *                   FP64) are passive.  skin is ignored when periodic. */
typedef struct sr_box {
    double len[3];
    int32_t periodic;
    int32_t _pad;
    double skin;
} sr_box;

typedef struct sr_ctx sr_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).
 *   arena_bytes > 0 : fixed scratch arena of that many bytes, allocated
 *                     here; calls needing more return SR_ENOMEM.
 *   arena_bytes == 0: the arena grows on demand.  The first call that
 *                     needs more waits for the stream, frees the old arena
 *                     and allocates 1.25x the need (a pool in the spirit of
 *                     the Bigchunk allocator of Sec. 2.7).
 * On success *out receives the context.  Returns SR_EINVAL / SR_EDEVICE /
 * SR_ENOMEM. */
int sr_ctx_create(int device, void *hip_stream, size_t arena_bytes, sr_ctx **out);

/* Wait for the context's stream, free the arena and the context. */
int sr_ctx_destroy(sr_ctx *ctx);

/* Message of the last error returned on this context ("" if none).  The
 * string is owned by the context and valid until its next call. */
const char *sr_last_error(const sr_ctx *ctx);

/* Change the stream later calls enqueue on.  Every call of a context shares
 * its scratch arena, so the new stream is made to wait (on the device, no
 * host wait) for the work already enqueued on the old one before anything
 * enqueued afterwards can start.  SR_EDEVICE if that ordering fails. */
int sr_set_stream(sr_ctx *ctx, void *hip_stream);

/* Bytes of arena currently allocated, and the high-water need so far. */
int sr_arena_info(const sr_ctx *ctx, size_t *allocated, size_t *high_water);

/* Wait for all work enqueued by this context; returns SR_ERANGE if a kernel
 * saw a coordinate outside [0, L) or a NaN, or sr_permute a perm entry
 * outside [0, n), since the last sr_sync (the results of such calls are
 * undefined but every access stayed in bounds),
 * SR_EDEVICE on a HIP error, else SR_OK.  Clears the device status. */
int sr_sync(sr_ctx *ctx);

/* Chaining-mesh geometry (host only, no device work): dims[d] =
 * floor(len[d] / cell) cells per axis, *n_cells = their product.  Cell
 * width cs_d = len[d] / dims[d] >= cell.  SR_EINVAL if cell <= 0, a side
 * is not positive, or a count overflows int32. */
int sr_grid_dims(const sr_box *box, double cell, int32_t dims[3], int64_t *n_cells);

/* Scratch bytes sr_force (with_force = 1) or sr_bin (0) needs for n
 * particles in this geometry; with_force = 2: an sr_ksk_step with multilevel
 * subcycles (its short-range passes with an activity mask, sub-item sums,
 * levels and counts).  A fixed arena of at least this size never returns
 * SR_ENOMEM for such a call.  Up to 2^22 particles a force pass may cut the
 * work of dense cells into sub-items whose partial sums take 112 bytes per
 * particle (about 210 bytes per particle in all; about 41 beyond). */
int sr_scratch_bytes(const sr_box *box, double cell, int64_t n, int with_force, size_t *bytes);

/* Chaining-mesh binning (a stable sort by cell: a counting sort, or for
 * n >= 2^22 an LSD radix sort of the cell ids, with the same result).
 *   x, y, z      : device float32[n], 0 <= coordinate < len.
 *   n            : 0 <= n <= 2^31 - 1.
 *   cell         : requested cell width (see sr_grid_dims).
 *   cell_offsets : device int32[n_cells + 1]; particles of cell c occupy
 *                  sorted slots [cell_offsets[c], cell_offsets[c+1]).
 *                  Cell of a coordinate: floor(x * (dims/len)) evaluated in
 *                  FP64 and clamped to dims-1; cell id = cx + dims[0]*(cy +
 *                  dims[1]*cz).
 *   perm         : device int32[n]; perm[k] = original index of sorted slot
 *                  k.  Within a cell, original order is kept (stable), so
 *                  the result is unique and deterministic.
 * This is the permutation array of Sec. 2.7 over the fixed short-range bins
 * of Sec. 3.1.  Errors: SR_EINVAL (null pointer with n > 0, bad geometry,
 * n out of range), SR_ENOMEM; SR_ERANGE later from sr_sync. */
int sr_bin(sr_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
           const sr_box *box, double cell, int32_t *cell_offsets, int32_t *perm);

/* Out-of-place re-ordering of one particle attribute by a permutation, the
 * attribute-at-a-time re-ordering that a permutation array allows (Sec. 2.7):
 * out[k] = in[perm[k]] for 0 <= k < n.
 *   perm       : device int32[n], a permutation of 0..n-1 (sr_bin's perm).
 *   in, out    : device arrays of n elements of elem_bytes each (4, 8 or 16:
 *                float or int32, double, float4); they must not overlap.
 * With one scratch array of the largest attribute a caller re-orders all its
 * attributes in turn.  Particles kept in the last binning's cell order make
 * the next binning cheaper (few distinct cells per block of the histogram).
 * Errors: SR_EINVAL synchronously (n < 0 or > 2^31 - 1, NULL pointer with
 * n > 0, another elem_bytes, in == out); a perm entry outside [0, n) writes
 * zero bytes to its slot and makes sr_sync return SR_ERANGE. */
int sr_permute(sr_ctx *ctx, const int32_t *perm, int64_t n, int32_t elem_bytes, const void *in,
               void *out);

/* Short-range accelerations (Eq. (force), Sec. 3.1) of all n particles.
 *   x, y, z, mass : device float32[n] (mass may be any finite values).
 *   cell          : chaining-mesh cell width; needs cs_d >= r_max and, in a
 *                   periodic box, dims[d] >= 3 and 2 r_max < len[d].
 *   r_max, eps    : cutoff radius (> 0) and softening (1e-20 <= eps), eps
 *                   added to s as in Eq. (force).
 *   poly          : HOST float[6], c_0..c_5 of p(s), read during the call.
 *   ax, ay, az    : device float32[n] outputs in the caller's original
 *                   particle order; passive particles get exactly 0.
 *   momentum3     : optional device double[3]; receives sum_i m_i a_i,
 *                   reduced in FP64 on the device in a fixed order (a Newton's
 *                   third law check; ~0 in a periodic box).
 * Arithmetic is float32 (one reciprocal square root per pair); each
 * target's sum is formed in tiles of at most 256 sources whose partial sums
 * are then added, and the result is deterministic (no floating-point atomics,
 * fixed order).  Errors: SR_EINVAL, SR_ENOMEM synchronously; SR_ERANGE from
 * sr_sync. */
int sr_force(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *mass,
             int64_t n, const sr_box *box, double cell, float r_max, float eps,
             const float poly[6], float *ax, float *ay, float *az, double *momentum3);

/* sr_force for callers that cannot allocate device memory while they run:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Arguments, outputs, errors and results are those of sr_force
 * (bitwise, at the same tuning); the difference is where the scratch lives.
 * Instead of the context arena (which sr_force may grow with hipMalloc) the
 * call uses one fixed device array of sr_force_static_capacity() bytes
 * (128 MiB) per GPU, held from the library's load until the process ends;
 * this call allocates nothing (no hipMalloc, no events, no library
 * allocation).  The scratch is sr_force's (sr_scratch_bytes with
 * with_force = 1): about 210 bytes per particle plus some per chaining cell
 * up to 2^22 particles, so that a box of 80^3 particles fits; a call needing
 * more returns SR_ENOMEM with a message and enqueues nothing.  No timing record
 * is taken (sr_timing_collect does not see these calls).
 * Concurrency: every call on one GPU shares that GPU's array, whatever its
 * context or stream, and the array keeps the last call's contents (each
 * call clears what it needs zeroed).  Calls that may overlap on one GPU --
 * on different streams, or from different threads -- race on it: serialize
 * them (one stream, or events between the streams). */
int sr_force_static(sr_ctx *ctx, const float *x, const float *y, const float *z,
                    const float *mass, int64_t n, const sr_box *box, double cell, float r_max,
                    float eps, const float poly[6], float *ax, float *ay, float *az,
                    double *momentum3);

/* Bytes of sr_force_static's fixed scratch array (per GPU). */
size_t sr_force_static_capacity(void);

/* Pair statistics for the same call shape as sr_force (no accelerations):
 *   *useful     : directed pairs (i, j), i != j, i not passive, with the
 *                 float32 s_ij < r_max^2 -- the interactions Eq. (force)
 *                 requires.
 *   *candidates : directed pairs the force loop evaluates: sum over
 *                 non-passive targets of the sources of their neighbour
 *                 cells that pass the work item's box test (sources whose
 *                 distance to the bounding box of the item's targets is
 *                 within r_max; the others cannot interact with any of
 *                 them).  Both counts use the work items of the current
 *                 tuning.
 *   per_target  : optional device int32[n]: useful partners of each particle
 *                 (original order).
 * *useful and *candidates are HOST pointers; this call waits for the
 * stream (it is a measurement helper, not part of the timed path). */
int sr_pair_stats(sr_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                  const sr_box *box, double cell, float r_max, int32_t *per_target,
                  int64_t *useful, int64_t *candidates);

/* Tuning of the pair loop (results are the same up to float32 summation
 * order for every setting; for a fixed setting they are bitwise
 * reproducible):
 *   xsplit     : 1..4 sub-cells per chaining cell along x.  The x-contiguous
 *                rows of the 27-cell search then span 2 + 1/xsplit chaining
 *                cells instead of 3, so fewer candidate pairs are tested; work
 *                items get smaller.  Default 1: with the box test of the
 *                pair loop (see sr_pair_stats), finer sub-cells save
 *                little more and cost more items.
 *   order      : 0 work items in cell order; 1 by decreasing cost bucket
 *                (longest first), default.
 *   persistent : 0 one workgroup per work item (default); 1 a fixed grid of
 *                workgroups takes items from a device counter.
 *   cell_scale : plans only (sr_plan_*): chaining cell = cell * cell_scale,
 *                >= 1; ignored by sr_set_tuning. */
typedef struct sr_tuning {
    int32_t xsplit;
    int32_t order;
    int32_t persistent;
    float cell_scale;
} sr_tuning;

int sr_set_tuning(sr_ctx *ctx, const sr_tuning *t);
int sr_get_tuning(const sr_ctx *ctx, sr_tuning *t);

/* ---- Precision form: split (cell + offset) coordinates ----------------- */

/* A coordinate x of a PERIODIC box meshed into dims = floor(len/cell) chaining
 * cells of width h = len/dims is held as its cell c = floor(x / h) (FP64) and
 * the float32 offset o = fl32(x - c h) in [0, h).  The three cell indices
 * are packed into one int32, cx | cy << 10 | cz << 20 (dims <= 1023 per
 * axis).  Offsets carry rounding of ulp(h) instead of ulp(len), and the pair
 * loop differences them without forming global coordinates, so float32
 * forces track float64 master positions more closely than global float32
 * coordinates can. */

/* float64 positions (device double[n], 0 <= x < len) -> split coordinates
 * (device int32 cell3[n], float ox/oy/oz[n]).  Out-of-range input sets the
 * device status (SR_ERANGE at sr_sync). */
int sr_split_from_f64(sr_ctx *ctx, const double *x, const double *y, const double *z, int64_t n,
                      const sr_box *box, double cell, int32_t *cell3, float *ox, float *oy,
                      float *oz);

/* Split coordinates -> float64 positions in [0, len). */
int sr_split_to_f64(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                    const float *oz, int64_t n, const sr_box *box, double cell, double *x,
                    double *y, double *z);

/* sr_force (Eq. (force), Sec. 3.1) on split coordinates: the same sum, with
 * every separation formed as (o_j + cell-offset shift) - o_i in float32.
 * Periodic boxes only; the x sub-cell count is min(tuning xsplit, 3).  An
 * offset outside [0, 1.0001 h] or a cell index out of range sets the device
 * status. */
int sr_force_split(sr_ctx *ctx, const int32_t *cell3, const float *ox, const float *oy,
                   const float *oz, const float *mass, int64_t n, const sr_box *box, double cell,
                   float r_max, float eps, const float poly[6], float *ax, float *ay, float *az,
                   double *momentum3);

/* One stream-kick-stream step (Sec. 2.5) of one periodic box held in split
 * coordinates, with the short-range force only:
 *   o += v dt/2 (FP64, re-homed);  a = sr_force_split;  v += a dt;
 *   o += v dt/2 (FP64, re-homed).
 * These are the maps of the serving form (sr_server_*): a box stepped by this
 * call follows bitwise the trajectory it follows inside a server with the
 * same cell and tuning.  cell3, ox, oy, oz, vx, vy, vz (device) are updated in
 * place; ax, ay, az (device float32[n]) receive the step's accelerations.
 * Arguments, scratch and errors as sr_force_split; dt finite. */
int sr_sks_split(sr_ctx *ctx, int32_t *cell3, float *ox, float *oy, float *oz, float *vx,
                 float *vy, float *vz, const float *mass, int64_t n, const sr_box *box,
                 double cell, float r_max, float eps, const float poly[6], float dt, float *ax,
                 float *ay, float *az);

/* ---- FP64 reductions on the device ------------------------------------ */

/* Kinetic energy K = sum_i m_i |v_i|^2 / 2 in FP64 (device float32 inputs,
 * *out a device double), reduced in a fixed order (bitwise reproducible).
 * The companion of the momentum sum that sr_force returns. */
int sr_kinetic(sr_ctx *ctx, const float *vx, const float *vy, const float *vz, const float *mass,
               int64_t n, double *out);

/* ---- RCB-tree variant (Sec. 2.4 RCB tree, Sec. 3.1 trees per fixed bin) - */

/* sr_force computed with an RCB tree inside every chaining cell instead of
 * whole-cell stencils.  A cell holding more than leaf_max particles is split
 * recursively by the plane through the centre of mass of a node (FP64,
 * mass-weighted) perpendicular to the longest side of its bounding box,
 * down to leaves of at most leaf_max particles (a node whose box is a point,
 * whose plane leaves a side empty, or 32 levels deep is a leaf whatever its
 * size).  Each leaf's particles share one interaction list: the leaves of
 * the 27 neighbouring cells whose bounding boxes come within r_max of the
 * leaf's box.  The sum is the same as sr_force's (every pair with
 * s < r_max^2), in a different order.  Arguments as sr_force, plus
 * leaf_max (1 .. 2^20); x sub-cells are not used.  Errors as sr_force. */
int sr_force_tree(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *mass,
                  int64_t n, const sr_box *box, double cell, float r_max, float eps,
                  const float poly[6], int32_t leaf_max, float *ax, float *ay, float *az,
                  double *momentum3);

/* The leaves sr_force_tree would use: leaf_of (device int32[n]) receives
 * the leaf index of every particle (leaves numbered cell by cell); the leaf
 * count is returned in *n_leaves (HOST; this call waits).  cell >= the
 * cutoff the caller will use. */
int sr_tree_leaves(sr_ctx *ctx, const float *x, const float *y, const float *z, const float *mass,
                   int64_t n, const sr_box *box, double cell, int32_t leaf_max, int32_t *leaf_of,
                   int64_t *n_leaves);

/* ---- Batched form: many independent boxes per pass -------------------- */

/* One box of a batch: device float32 inputs and outputs of its own, its own
 * geometry and chaining cell.  Boxes never interact.
 *   cell3 == NULL : x, y, z are global coordinates (as sr_force).
 *   cell3 != NULL : split coordinates of a periodic box (as sr_force_split):
 *                   cell3 holds the packed chaining cells of the mesh given
 *                   by `cell` and x, y, z the float32 offsets.  Such a box
 *                   needs cell_scale 1 and uses min(xsplit, 3) x sub-cells. */
typedef struct sr_batch_box {
    const float *x, *y, *z, *mass;
    int64_t n;
    sr_box box;
    double cell;
    float *ax, *ay, *az;
    const int32_t *cell3;
} sr_batch_box;

typedef struct sr_plan sr_plan;

/* A plan evaluates Eq. (force) for all boxes of a batch in one pass: one
 * segmented binning over the concatenated cell space, one pair-loop launch
 * over every box's work items (longest first), and per-box FP64 momentum.
 * (The paper's GPU design makes independent blocks the unit of work, Sec.
 * 3.3; here a batch of boxes is one launch.)
 *   boxes      : nboxes descriptors (HOST array, copied; device pointers
 *                inside must stay valid for the plan's lifetime).  Each box
 *                obeys the sr_force rules; total particles <= 2^31 - 1.
 *   r_max, eps, poly : as sr_force, shared by all boxes.
 *   momentum   : optional device double[3 * nboxes]; box b's sum_i m_i a_i
 *                lands in momentum[3b .. 3b+2].
 * The plan owns its scratch (sized for every tuning) and its descriptor
 * table; creation waits for the upload.  Each box's accelerations are
 * bitwise those of sr_force (sr_force_split for a box with cell3) on that
 * box alone with the same sr_tuning.
 * Errors: SR_EINVAL (a bad box, with its index in sr_last_error),
 * SR_ENOMEM, SR_EDEVICE. */
int sr_plan_create(sr_ctx *ctx, const sr_batch_box *boxes, int nboxes, float r_max, float eps,
                   const float poly[6], double *momentum, sr_plan **out);

/* Change the plan's tuning (xsplit, order, persistent, cell_scale >= 1);
 * re-uploads the descriptors (waits) and drops a captured graph.
 * SR_EINVAL if some box is invalid at that cell_scale. */
int sr_plan_set_tuning(sr_plan *plan, const sr_tuning *t);
int sr_plan_get_tuning(const sr_plan *plan, sr_tuning *t);

/* Enqueue one pass on the plan's stream (the context's stream, or a stream
 * of the plan's own when the context uses the legacy default stream). */
int sr_plan_run(sr_plan *plan);

/* Record one pass into a HIP graph (no allocation, no memset nodes, no host
 * synchronisation inside); sr_plan_launch then replays it.  The graph reads
 * the boxes' current input buffers at every replay. */
int sr_plan_capture(sr_plan *plan);

/* Replay the captured graph (captures first if needed). */
int sr_plan_launch(sr_plan *plan);

/* Project autotuner: times `reps` passes (after one warm-up) of every
 * candidate tuning -- xsplit in {1, 2, 3}, order in {0, 1}, persistent in
 * {0, 1}, cell_scale in {1, 1.25} -- with HIP events, keeps the fastest
 * (median), and leaves the plan set to it.  best / best_ms are HOST
 * pointers (either may be NULL).  Waits for the stream. */
int sr_plan_autotune(sr_plan *plan, int reps, sr_tuning *best, double *best_ms);

/* Wait for the plan's stream and free everything the plan owns. */
int sr_plan_destroy(sr_plan *plan);

/* ---- Serving form: continuous batching of time-stepping requests ------- */

/* A request evolves one periodic cube of n particles for `steps`
 * stream-kick-stream steps (Sec. 2.5: x += v dt/2; a = f_SR; v += a dt;
 * x += v dt/2) with the short-range force only.  State stays resident in
 * HBM in split coordinates (cell + float32 offset, velocity float32) from
 * admission to completion. */
typedef struct sr_request {
    int64_t n;
    double len;                  /* cube side; must be exact in float32 */
    int32_t steps;               /* >= 1 */
    float dt;
    const double *x, *y, *z;     /* HOST float64 initial positions in [0, len) */
    const float *vx, *vy, *vz;   /* HOST initial velocities */
    const float *mass;           /* HOST masses */
    double *out_x, *out_y, *out_z;   /* HOST final positions (written at completion) */
    float *out_vx, *out_vy, *out_vz; /* HOST final velocities */
    double *out_kinetic;             /* HOST, optional: FP64 sum m |v|^2 / 2 of the final state */
} sr_request;

typedef struct sr_server_config {
    size_t hbm_budget;     /* bytes: half for resident state, half for pass scratch */
    int32_t max_slots;     /* requests active at once (1 .. 131072) */
    float r_max, eps;
    float poly[6];
    double cell;           /* chaining cell of every request's box */
    sr_tuning tuning;      /* xsplit (<= 3 used), order, persistent; fixed for the server */
} sr_server_config;

typedef struct sr_server_info {
    int64_t queued, active, draining, completed;
    size_t state_bytes_in_use, state_bytes_high_water, state_bytes_capacity;
    size_t scratch_bytes_capacity;
    int64_t ticks;
} sr_server_info;

typedef struct sr_server sr_server;

/* Create a server on the context's device and stream; allocates the budget
 * up front (one state pool, one scratch arena).  Errors: SR_EINVAL,
 * SR_ENOMEM. */
int sr_server_create(sr_ctx *ctx, const sr_server_config *cfg, sr_server **out);

/* Queue a request (FIFO).  The host arrays it points to must stay valid until
 * the request completes (outputs should be pinned host memory so that the
 * result copies stay asynchronous).  *id receives the request id.
 * SR_EINVAL for an invalid request, SR_EBUSY if the request could never fit
 * the budget. */
int sr_server_submit(sr_server *srv, const sr_request *req, int64_t *id);

/* One tick: admit queued requests in order while slots, state memory and
 * scratch allow; advance every active request by one step in a single
 * batched pass (stream, binning, pair loop, kick + stream); start the result
 * copies of requests that finished.  Only enqueues work, except that it may
 * wait for the tick that used the same descriptor buffer R ticks ago.
 * *active (HOST, may be NULL) receives the number of requests stepped. */
int sr_server_tick(sr_server *srv, int *active);

/* Ids of requests whose results have landed in their host outputs since the
 * last poll (HOST array of capacity cap; *n receives the count).  Frees their
 * state memory. */
int sr_server_poll(sr_server *srv, int64_t *ids, int cap, int *n);

/* Drop a queued or active request; its memory is freed once the device no
 * longer uses it.  Other requests are unaffected.  SR_EINVAL if unknown or
 * already finished. */
int sr_server_cancel(sr_server *srv, int64_t id);

int sr_server_info_get(const sr_server *srv, sr_server_info *info);

/* Wait for all work and free the server (requests still queued or active
 * are dropped). */
int sr_server_destroy(sr_server *srv);

/* Device-side timing of sr_force (a measurement helper).  While enabled,
 * each sr_force call records HIP events on the context's stream: one before
 * its preparation (binning, gather, work items), one before the pair-loop
 * kernel and one after it. */
int sr_timing_enable(sr_ctx *ctx, int enable);

/* Waits for the stream and returns, summed over the sr_force calls recorded
 * since the previous collect, the milliseconds of the preparation phase and
 * of the pair-loop kernel, and the number of calls (HOST pointers; any may
 * be NULL).  Resets the record. */
int sr_timing_collect(sr_ctx *ctx, double *prep_ms, double *force_ms, int64_t *calls);

#ifdef __cplusplus
}
#endif
#endif /* SR_H */
