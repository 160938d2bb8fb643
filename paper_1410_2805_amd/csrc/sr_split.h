// Split coordinates and the serving state update (sr_split.hip).
#pragma once

#include "sr_internal.h"

// Chaining-mesh geometry of split coordinates: h = len / nc, FP64.
struct SplitGeom {
    double len[3];
    double inv[3];
    double h[3];
    int nc[3];
    int _pad;
};

// One serving slot: resident split state of one box (device pointers).

struct SlotState {
    SplitGeom g;
    float dt;
    int _pad;
    int *cell3;
    float *ox, *oy, *oz;
    float *vx, *vy, *vz;
    const float *ax, *ay, *az;
};

int split_geom(sr_ctx *ctx, const sr_box *box, double cell, SplitGeom *sg);
int split_from_f64_enqueue(sr_ctx *ctx, const double *x, const double *y, const double *z, int n,
                           const SplitGeom &sg, int *cell3, float *ox, float *oy, float *oz);
int split_to_f64_enqueue(sr_ctx *ctx, const int *cell3, const float *ox, const float *oy,
                         const float *oz, int n, const SplitGeom &sg, double *x, double *y,
                         double *z);
// mode 0: stream half step; mode 1: kick then stream half step.
int slot_update_enqueue(sr_ctx *ctx, const SlotState *slots, const int *start, int nslot,
                        int ntot, int mode);
// One box: v += a * kick (a may be null: no kick), then nstream times
// o += v * stream in FP64 with re-homing (stream == 0: no stream); two
// streams are bitwise two calls with one.
int kick_stream_enqueue(sr_ctx *ctx, const SplitGeom &sg, int n, int *cell3, float *ox, float *oy,
                        float *oz, float *vx, float *vy, float *vz, const float *ax,
                        const float *ay, const float *az, float kick, double stream,
                        int nstream = 1);

// Multilevel stepping (Sec. 3.1, Eq. (kicks)) on one box of split state.
// level[i] = clamp(floor(count * ncell / n) / d + 1, lmin, lmax) from the
// chaining-cell counts (counts: ncell ints of scratch).
int ml_levels_enqueue(sr_ctx *ctx, const SplitGeom &sg, const int *cell3, int n, int *counts,
                      int d, int lmin, int lmax, unsigned char *level);
// active[i] = 1 where level[i] kicks after stream piece m of M (2 when
// level[i] > lmin: the pass cuts such particles' cells into finer items).
int ml_active_enqueue(sr_ctx *ctx, const unsigned char *level, int n, int m, int M, int lmin,
                      unsigned char *active);
// Kick the particles whose level kicks at m by a tau / level (a may be null),
// then stream every particle nstream times by `stream` (0: none), rounding
// after each as separate pieces would.
int ml_update_enqueue(sr_ctx *ctx, const SplitGeom &sg, int n, int *cell3, float *ox, float *oy,
                      float *oz, float *vx, float *vy, float *vz, const float *ax,
                      const float *ay, const float *az, const unsigned char *level, int m, int M,
                      double tau, double stream, int nstream);

// FP64 K = sum m |v|^2 / 2 into *out (device); part: kRedBlocks doubles.
int kinetic_enqueue(sr_ctx *ctx, const float *vx, const float *vy, const float *vz,
                    const float *m, int n, double *part, double *out);
