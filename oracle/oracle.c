/*
 * FP64 reference ("oracle") for the short-range particle-particle force of the
 * HACC hybrid N-body method (Habib et al., "HACC: Simulating Sky Surveys on
 * State-of-the-Art Supercomputing Architectures", arXiv:1410.2805).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Each function is the plain definition, written out in double precision and
 * evaluated the slow, obvious way:
 *
 *   oracle_grid_dims  chaining-mesh geometry: cells no smaller than the cell
 *                     size asked for (Sec. 2.4, last paragraph: the chaining
 *                     mesh of P3M; Sec. 3.1: fixed bins of about the
 *                     short-range scale, searched with their 26 neighbours).
 *   oracle_bin        particle -> cell id, then a stable counting sort that
 *                     yields the cell offsets and the permutation array
 *                     (Sec. 2.7: a permuted ordering of the particles used to
 *                     reorder each attribute out of place).
 *   oracle_force      Eq. (force) of Sec. 3.1, f_SR(s) = (s+eps)^(-3/2) - p(s),
 *                     p a fifth-order polynomial in s = r.r standing for the
 *                     grid force of Sec. 2.4, summed over every pair closer
 *                     than r_max by an O(N) scan of all sources per target.
 *                     Passive particles of an overloaded (non-periodic)
 *                     domain get no short-range force (Sec. 2.2).
 *   oracle_sks        one stream-kick-stream step (Sec. 2.5) with that force.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - p multiplies the separation vector, so it is the grid force divided by
 *     r; the acceleration on i is sum_j m_j f_SR(s_ij) (x_j - x_i), G = 1 in
 *     code units (Sec. 2.6), pointing from i towards j.
 *   - eps is added to s (a squared length), exactly as Eq. (force) reads.
 *   - the cutoff is strict: pairs with s < r_max^2 interact.
 *   - periodic boxes use the minimum image of x_j - x_i.
 *   - a particle is passive when its distance to the nearest face of a
 *     non-periodic box is below the skin width (strict), computed in FP64.
 *   - cell of a coordinate: floor(x * (n_c / L)) in FP64, clamped to n_c - 1;
 *     linear cell id cx + n_cx (cy + n_cy cz) (x fastest).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-22)
#define ORACLE_ERANGE (-34)
#define ORACLE_ENOMEM (-12)

/* Number of cells per side: the largest count whose cells are still at least
 * `cell` wide, n_c = floor(L / cell). */
int oracle_grid_dims(const double L[3], double cell, int32_t nc[3])
{
    if (!(cell > 0.0))
        return ORACLE_EINVAL;
    for (int d = 0; d < 3; ++d) {
        if (!(L[d] > 0.0))
            return ORACLE_EINVAL;
        double q = floor(L[d] / cell);
        if (q < 1.0 || q > 2147483647.0)
            return ORACLE_EINVAL;
        nc[d] = (int32_t)q;
    }
    return ORACLE_OK;
}

static int32_t cell_coord(double x, double L, int32_t nc)
{
    double inv = (double)nc / L;
    double t = floor(x * inv);
    int32_t c = (int32_t)t;
    if (c > nc - 1)
        c = nc - 1;
    if (c < 0)
        c = 0;
    return c;
}

/* Stable counting sort of particles by cell id.
 *   x, y, z   : n positions (float32 values promoted to double), 0 <= x < L
 *   offsets   : n_cells + 1 entries; particles of cell c are sorted slots
 *               [offsets[c], offsets[c+1])
 *   perm      : n entries; perm[k] is the original index of sorted slot k;
 *               equal cells keep their original relative order
 *   cid       : optional, n entries; cell id of each original particle
 * Returns ORACLE_ERANGE (and *bad = index) when a coordinate lies outside
 * [0, L) or is NaN. */
int oracle_bin(const double *x, const double *y, const double *z, int64_t n,
               const double L[3], double cell, int32_t *offsets, int32_t *perm,
               int32_t *cid, int64_t *bad)
{
    int32_t nc[3];
    int rc = oracle_grid_dims(L, cell, nc);
    if (rc)
        return rc;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *count = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    if (!id || !count) {
        free(id);
        free(count);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int d = 0; d < 3; ++d) {
            if (!(p[d] >= 0.0 && p[d] < L[d])) {
                if (bad)
                    *bad = i;
                free(id);
                free(count);
                return ORACLE_ERANGE;
            }
        }
        int32_t cx = cell_coord(p[0], L[0], nc[0]);
        int32_t cy = cell_coord(p[1], L[1], nc[1]);
        int32_t cz = cell_coord(p[2], L[2], nc[2]);
        id[i] = cx + nc[0] * (cy + nc[1] * cz);
        count[id[i]] += 1;
    }
    /* exclusive prefix sum of the histogram */
    int64_t run = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t k = count[c];
        offsets[c] = (int32_t)run;
        count[c] = run; /* reused as the write cursor of cell c */
        run += k;
    }
    offsets[ncell] = (int32_t)run;
    /* scatter in increasing original index: this is what makes it stable */
    for (int64_t i = 0; i < n; ++i)
        perm[count[id[i]]++] = (int32_t)i;
    if (cid)
        memcpy(cid, id, sizeof(int32_t) * (size_t)n);
    free(id);
    free(count);
    return ORACLE_OK;
}

static double poly5(const double c[6], double s)
{
    /* p(s) = c0 + c1 s + c2 s^2 + c3 s^3 + c4 s^4 + c5 s^5 */
    double acc = 0.0, sk = 1.0;
    for (int k = 0; k < 6; ++k) {
        acc += c[k] * sk;
        sk *= s;
    }
    return acc;
}

static int is_passive(const double p[3], const double L[3], int periodic, double skin)
{
    if (periodic)
        return 0;
    for (int d = 0; d < 3; ++d) {
        double lo = p[d];
        double hi = L[d] - p[d];
        if (lo < skin || hi < skin)
            return 1;
    }
    return 0;
}

/* Short-range accelerations by brute force over all sources.
 *
 *   x, y, z, m : n sources (and candidate targets), double
 *   L          : box sides; periodic != 0 selects the minimum image
 *   skin       : passive-skin width, used only when periodic == 0
 *   r_max, eps : cutoff radius and Plummer softening (added to s)
 *   poly       : c_0..c_5 of p(s)
 *   targets    : nt target indices, or NULL for all n particles in order
 * Outputs, one entry per target (any may be NULL):
 *   ax, ay, az : a_i = sum_{j != i, s_ij < r_max^2} m_j f_SR(s_ij) d_ij
 *   sabs       : S_i = sum of |m_j f_SR(s_ij)| |d_ij| over the same pairs
 *   tie        : A_i = sum of |m_j f_SR(s_ij)| |d_ij| over pairs j != i with
 *                |s_ij - r_max^2| <= 2^-18 r_max^2 (on either side of the
 *                cutoff): pairs a float32 evaluation of s may classify
 *                differently from the exact one
 *   npair      : number of j != i with s_ij < r_max^2 (0 for passive i)
 *   passive    : 1 if target is passive (accelerations are then exactly 0)
 * nthreads <= 0 uses the OpenMP default. */
int oracle_force(const double *x, const double *y, const double *z, const double *m,
                 int64_t n, const double L[3], int periodic, double skin, double r_max,
                 double eps, const double poly[6], const int64_t *targets, int64_t nt,
                 double *ax, double *ay, double *az, double *sabs, double *tie,
                 int64_t *npair, int32_t *passive, int nthreads)
{
    if (!(eps >= 0.0) || !(r_max > 0.0))
        return ORACLE_EINVAL;
    if (periodic)
        for (int d = 0; d < 3; ++d)
            if (!(2.0 * r_max < L[d]))
                return ORACLE_EINVAL;
    const double r2 = r_max * r_max;
    const double band = r2 * ldexp(1.0, -18);
    if (!targets)
        nt = n;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        const double pi[3] = {x[i], y[i], z[i]};
        double a[3] = {0.0, 0.0, 0.0};
        double S = 0.0, A = 0.0;
        int64_t cnt = 0;
        const int pas = is_passive(pi, L, periodic, skin);
        if (!pas) {
            for (int64_t j = 0; j < n; ++j) {
                if (j == i)
                    continue;
                double d[3] = {x[j] - pi[0], y[j] - pi[1], z[j] - pi[2]};
                if (periodic) {
                    for (int k = 0; k < 3; ++k) {
                        if (d[k] > 0.5 * L[k])
                            d[k] -= L[k];
                        else if (d[k] < -0.5 * L[k])
                            d[k] += L[k];
                    }
                }
                double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                int near_cut = fabs(s - r2) <= band;
                if (!(s < r2) && !near_cut)
                    continue;
                double se = s + eps;
                double f = 1.0 / (se * sqrt(se)) - poly5(poly, s);
                double w = m[j] * f;
                double mag = fabs(w) * sqrt(s);
                if (near_cut)
                    A += mag;
                if (s < r2) {
                    a[0] += w * d[0];
                    a[1] += w * d[1];
                    a[2] += w * d[2];
                    S += mag;
                    cnt += 1;
                }
            }
        }
        if (ax) ax[t] = a[0];
        if (ay) ay[t] = a[1];
        if (az) az[t] = a[2];
        if (sabs) sabs[t] = S;
        if (tie) tie[t] = A;
        if (npair) npair[t] = cnt;
        if (passive) passive[t] = pas;
    }
    return ORACLE_OK;
}

/* Maximum-threads query for reporting the core count actually used. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One stream-kick-stream step (Sec. 2.5) of every particle of a periodic box:
 *   x += v dt/2 (wrapped into [0, L));  a = short-range force;
 *   v += a dt;  x += v dt/2 (wrapped).
 * Positions and velocities are double "master" state; acc (n x 3, may be
 * NULL) receives the accelerations used for the kick. */
int oracle_sks(double *x, double *y, double *z, double *vx, double *vy, double *vz,
               const double *m, int64_t n, const double L[3], double r_max, double eps,
               const double poly[6], double dt, double *acc, int nthreads)
{
    double *P[3] = {x, y, z};
    double *V[3] = {vx, vy, vz};
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
            double u = P[d][i] + 0.5 * dt * V[d][i];
            u -= L[d] * floor(u / L[d]);
            if (u >= L[d]) u -= L[d];
            P[d][i] = u;
        }
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!a)
        return ORACLE_ENOMEM;
    int rc = oracle_force(x, y, z, m, n, L, 1, 0.0, r_max, eps, poly, NULL, n, a, a + n,
                          a + 2 * n, NULL, NULL, NULL, NULL, nthreads);
    if (rc) {
        free(a);
        return rc;
    }
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) {
            V[d][i] += dt * a[d * n + i];
            double u = P[d][i] + 0.5 * dt * V[d][i];
            u -= L[d] * floor(u / L[d]);
            if (u >= L[d]) u -= L[d];
            P[d][i] = u;
        }
    if (acc)
        memcpy(acc, a, sizeof(double) * 3 * (size_t)n);
    free(a);
    return ORACLE_OK;
}
