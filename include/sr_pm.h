/* Long-range particle-mesh (PM) force and the subcycled full step.
 *
 * The long-range solver of Sec. 2.3: cloud-in-cell (CIC) deposit of the
 * masses on a periodic N_g^3 grid, one forward 3-D FFT, the composition in
 * k space of the sinc-Gaussian filter (Eq. (filter)), the sixth-order
 * influence function (Eq. (greenf)) and the fourth-order Super-Lanczos
 * gradient (Eq. (sldiff)), inverse FFTs, and CIC interpolation of the
 * gradient back to the particles.  G = 1 (Sec. 2.6); lengths are in any unit
 * with the grid spacing Delta = len / N_g, the filter width sigma is given in
 * grid spacings, and grid point (i, j, k) sits at (i, j, k) Delta.
 *
 * Conventions shared with sr.h: every pointer argument that names particle or
 * grid data is a DEVICE pointer on the context's device; calls enqueue on the
 * context's stream and return without waiting; invalid arguments return
 * SR_EINVAL synchronously, and data errors found by a kernel (a negative or
 * non-finite mass, a non-finite position) are reported as SR_ERANGE by the
 * next sr_sync.  Nothing here allocates after creation.
 *
 * Grids are stored x-major (index (i N_g + j) N_g + k, k fastest).
 */
#ifndef SR_PM_H
#define SR_PM_H

#include "sr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sr_pm sr_pm;

/* Create a PM solver for a periodic cube of side len with an ng^3 grid, bound
 * to ctx (its device and stream).  ng must be a power of two in [8, 1024];
 * sigma > 0 (grid spacings) and ns >= 0 are the filter parameters of Eq.
 * (filter) (nominal 0.8 and 3).  The solver owns two complex float32 grids
 * and a 64-bit deposit grid (24 ng^3 bytes) and its k-space tables, built in
 * FP64 on the host and uploaded before this call returns.  Errors: SR_EINVAL, SR_ENOMEM,
 * SR_EDEVICE. */
int sr_pm_create(sr_ctx *ctx, int32_t ng, double len, float sigma, int32_t ns, sr_pm **out);

/* Free the solver's device memory (waits for the context's stream). */
int sr_pm_destroy(sr_pm *pm);

/* Device bytes a solver with this grid holds. */
int sr_pm_bytes(int32_t ng, size_t *bytes);

/* CIC mass density (mass / Delta^3) of n particles with float32 positions
 * x, y, z (any finite value; wrapped periodically) and masses >= 0, written
 * to rho (device float[ng^3]).  The deposit accumulates in 64-bit fixed point
 * with a quantum of 2^-S times the largest mass (S = 62 - ceil log2 max m -
 * ceil log2 n), so the result does not depend on the order of arrival and is
 * bitwise reproducible. */
int sr_pm_deposit(sr_pm *pm, const float *x, const float *y, const float *z, const float *mass,
                  int64_t n, float *rho);

/* In-place unnormalised 3-D DFT of data (device float[2 ng^3], interleaved
 * complex, grid order as above): X(k) = sum_j x(j) exp(-+2 pi i j.k / ng),
 * minus sign when inverse == 0.  The transform the solver uses internally
 * (radix-4/2 Stockham passes along each axis). */
int sr_pm_fft(sr_pm *pm, float *data, int32_t inverse);

/* Long-range accelerations (Sec. 2.3) of n particles on themselves and each
 * other: ax, ay, az (device float[n]) are overwritten.  Positions and masses
 * as sr_pm_deposit. */
int sr_pm_force(sr_pm *pm, const float *x, const float *y, const float *z, const float *mass,
                int64_t n, float *ax, float *ay, float *az);

/* sr_pm_force on split coordinates (sr.h) of a periodic cubic box of side
 * len (the solver's) meshed with chaining cell `cell`: position = c h + o in
 * FP64 with h = len / floor(len / cell). */
int sr_pm_force_split(sr_pm *pm, const int32_t *cell3, const float *ox, const float *oy,
                      const float *oz, const float *mass, int64_t n, double cell, float *ax,
                      float *ay, float *az);

/* Parameters of one full step of Eq. (tstep). */
typedef struct sr_step_params {
    float r_max, eps;   /* short-range cutoff and softening (sr_force) */
    float poly[6];      /* grid-force polynomial (sr_force) */
    double cell;        /* chaining cell of the split coordinates */
    float dt;           /* full step length */
    int32_t n_sub;      /* short-range subcycles per step (>= 1) */
    /* Multilevel subcycles (Sec. 3.1, Eq. (kicks)); ml_d = 0: off.  At the
     * start of each subcycle a particle gets l = floor(rho/rho_0) / ml_d + 1
     * kicks (integer division; rho/rho_0 = its chaining cell's count over
     * the mean count), clamped to [ml_min, ml_max] (1 <= ml_min <= ml_max <= 4).
     * Every particle streams in M = 2 lcm(ml_min..ml_max) pieces of tau/M; a
     * particle of level l kicks by tau/l after the pieces m with 2 m l / M
     * odd, with the short-range force evaluated for the cells holding such
     * particles. */
    int32_t ml_d, ml_min, ml_max;
} sr_step_params;

/* One full step of Eq. (tstep) (Sec. 2.5) on resident split state of a
 * periodic cube whose side is the solver's len:
 *   v += a_lr dt/2;  n_sub times { x += v tau/2; a_sr = sr_force_split;
 *   v += a_sr tau; x += v tau/2 } with tau = dt / n_sub;  a_lr = PM force at
 *   the new positions;  v += a_lr dt/2.
 * cell3, ox, oy, oz, vx, vy, vz are updated in place (positions are streamed
 * in FP64 and re-homed to their cells).  lr_ax/ay/az (device float[n]) hold
 * the PM acceleration: read as the value at the incoming positions when
 * lr_valid != 0 (the previous step's output), else computed first; on return
 * they hold it at the outgoing positions.  sr_ax/ay/az (device float[n])
 * receive the last subcycle's short-range acceleration (multilevel: each
 * particle's value from the last evaluation that covered its cell).  Tuning
 * and scratch come from the context as for sr_force_split (multilevel adds
 * 2 n + 4 n_cells bytes).  Errors: SR_EINVAL (box not a
 * periodic cube of the solver's side, bad parameters), SR_ENOMEM; SR_ERANGE
 * from sr_sync. */
int sr_ksk_step(sr_ctx *ctx, sr_pm *pm, int32_t *cell3, float *ox, float *oy, float *oz,
                float *vx, float *vy, float *vz, const float *mass, int64_t n,
                const sr_box *box, const sr_step_params *p, float *lr_ax, float *lr_ay,
                float *lr_az, int32_t lr_valid, float *sr_ax, float *sr_ay, float *sr_az);

#ifdef __cplusplus
}
#endif

#endif /* SR_PM_H */
