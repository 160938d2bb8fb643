// The full step of Eq. (tstep) (Sec. 2.5): long-range half kicks around
// n_sub short-range stream-kick-stream subcycles, on resident split state.
#include <climits>
#include <cmath>

#include "sr_internal.h"
#include "sr_pm.h"
#include "sr_split.h"

// sr_pm.hip
int pm_force_split_enqueue(sr_pm *pm, const int32_t *cell3, const float *ox, const float *oy,
                           const float *oz, const float *mass, int n, const double h[3],
                           float *ax, float *ay, float *az);
sr_ctx *pm_context(const sr_pm *pm);
double pm_len(const sr_pm *pm);

extern "C" int sr_ksk_step(sr_ctx *ctx, sr_pm *pm, int32_t *cell3, float *ox, float *oy,
                           float *oz, float *vx, float *vy, float *vz, const float *mass,
                           int64_t n, const sr_box *box, const sr_step_params *p, float *lr_ax,
                           float *lr_ay, float *lr_az, int32_t lr_valid, float *sr_ax,
                           float *sr_ay, float *sr_az)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (!pm || pm_context(pm) != ctx)
        return sr_fail(ctx, SR_EINVAL, "the PM solver must belong to this context");
    if (!box || !p)
        return sr_fail(ctx, SR_EINVAL, "NULL box or parameters");
    const double len = pm_len(pm);
    if (!box->periodic || box->len[0] != len || box->len[1] != len || box->len[2] != len)
        return sr_fail(ctx, SR_EINVAL, "the box must be the PM solver's periodic cube");
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n out of range");
    if (n > 0 && (!cell3 || !ox || !oy || !oz || !vx || !vy || !vz || !mass || !lr_ax ||
                  !lr_ay || !lr_az || !sr_ax || !sr_ay || !sr_az))
        return sr_fail(ctx, SR_EINVAL, "NULL pointer with n > 0");
    if (p->n_sub < 1 || !std::isfinite(p->dt))
        return sr_fail(ctx, SR_EINVAL, "n_sub must be >= 1 and dt finite");
    const bool ml = p->ml_d > 0;
    if (p->ml_d < 0 || (ml && !(1 <= p->ml_min && p->ml_min <= p->ml_max && p->ml_max <= 4)))
        return sr_fail(ctx, SR_EINVAL, "multilevel needs ml_d >= 0 and 1 <= ml_min <= ml_max <= 4");
    SplitGeom sg;
    int rc = split_geom(ctx, box, p->cell, &sg);
    if (rc)
        return rc;
    if ((rc = check_force_params(ctx, p->r_max, p->eps, p->poly)))
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    const int ni = (int)n;
    // multilevel scratch sits after the force pass's part of the arena
    unsigned char *level = nullptr, *active = nullptr;
    int *counts = nullptr;
    if (ml) {
        // sized for a masked pass (finer items, sub-item sums); the sizing
        // call only tests the mask pointer for null
        static const unsigned char any_mask = 1;
        size_t fbytes = 0;
        if ((rc = force_split_masked(ctx, cell3, ox, oy, oz, mass, n, box, p->cell, p->r_max,
                                     p->eps, p->poly, sr_ax, sr_ay, sr_az, nullptr, &any_mask,
                                     &fbytes)))
            return rc;
        const size_t a = 256;
        const size_t ncell = (size_t)sg.nc[0] * sg.nc[1] * sg.nc[2];
        const size_t off_level = (fbytes + a - 1) / a * a;
        const size_t off_active = off_level + ((size_t)n + a - 1) / a * a;
        const size_t off_counts = off_active + ((size_t)n + a - 1) / a * a;
        if ((rc = sr_arena_reserve(ctx, off_counts + ncell * sizeof(int))))
            return rc;
        level = reinterpret_cast<unsigned char *>(ctx->arena + off_level);
        active = reinterpret_cast<unsigned char *>(ctx->arena + off_active);
        counts = reinterpret_cast<int *>(ctx->arena + off_counts);
    }
    if (!lr_valid &&
        (rc = pm_force_split_enqueue(pm, cell3, ox, oy, oz, mass, ni, sg.h, lr_ax, lr_ay, lr_az)))
        return rc;
    const double tau = (double)p->dt / p->n_sub;
    const double half_tau = 0.5 * tau;
    const float half_dt = (float)(0.5 * (double)p->dt);
    if (ml) {
        int M = 1;
        for (int l = p->ml_min; l <= p->ml_max; ++l) {
            int g = M, b = l;
            while (b) {
                const int t = g % b;
                g = b;
                b = t;
            }
            M = M / g * l;
        }
        M *= 2;
        if ((rc = kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, lr_ax, lr_ay,
                                      lr_az, half_dt, 0.0)))
            return rc;
        const double piece = tau / M;
        auto kicks_at = [&](int m) {
            for (int l = p->ml_min; l <= p->ml_max; ++l)
                if ((2 * m * l) % M == 0 && ((2 * m * l / M) & 1))
                    return true;
            return false;
        };
        // pieces streamed after piece m up to the next kick time (or the end
        // of the subcycle), in one launch: nothing kicks in between
        auto streams_after = [&](int m) {
            int k = 0;
            for (int q = m; q < M && (q == m || !kicks_at(q)); ++q)
                ++k;
            return k;
        };
        for (int c = 0; c < p->n_sub; ++c) {
            if ((rc = ml_levels_enqueue(ctx, sg, cell3, ni, counts, p->ml_d, p->ml_min, p->ml_max,
                                        level)) ||
                (rc = ml_update_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, nullptr,
                                        nullptr, nullptr, level, 0, M, tau, piece,
                                        streams_after(0))))
                return rc;
            for (int m = 1; m <= M; ++m) {
                if (!kicks_at(m))
                    continue;  // its stream piece went with the last kick's launch
                const int ns = streams_after(m);
                if ((rc = ml_active_enqueue(ctx, level, ni, m, M, p->ml_min, active)) ||
                    (rc = force_split_masked(ctx, cell3, ox, oy, oz, mass, n, box, p->cell,
                                             p->r_max, p->eps, p->poly, sr_ax, sr_ay, sr_az,
                                             nullptr, active, nullptr)) ||
                    (rc = ml_update_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, sr_ax,
                                            sr_ay, sr_az, level, m, M, tau, ns ? piece : 0.0,
                                            ns)))
                    return rc;
            }
        }
        if ((rc = pm_force_split_enqueue(pm, cell3, ox, oy, oz, mass, ni, sg.h, lr_ax, lr_ay,
                                         lr_az)))
            return rc;
        return kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, lr_ax, lr_ay,
                                   lr_az, half_dt, 0.0);
    }
    // long-range half kick fused with the first subcycle's first stream
    if ((rc = kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, lr_ax, lr_ay, lr_az,
                                  half_dt, half_tau)))
        return rc;
    for (int c = 0; c < p->n_sub; ++c) {
        if ((rc = sr_force_split(ctx, cell3, ox, oy, oz, mass, n, box, p->cell, p->r_max, p->eps,
                                 p->poly, sr_ax, sr_ay, sr_az, nullptr)))
            return rc;
        // the kick, this subcycle's last half stream and, before another
        // subcycle, the next one's first half stream: one launch
        if ((rc = kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, sr_ax, sr_ay,
                                      sr_az, (float)tau, half_tau, c + 1 < p->n_sub ? 2 : 1)))
            return rc;
    }
    if ((rc = pm_force_split_enqueue(pm, cell3, ox, oy, oz, mass, ni, sg.h, lr_ax, lr_ay, lr_az)))
        return rc;
    return kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, lr_ax, lr_ay, lr_az,
                               half_dt, 0.0);
}

extern "C" int sr_sks_split(sr_ctx *ctx, int32_t *cell3, float *ox, float *oy, float *oz,
                            float *vx, float *vy, float *vz, const float *mass, int64_t n,
                            const sr_box *box, double cell, float r_max, float eps,
                            const float poly[6], float dt, float *ax, float *ay, float *az)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    if (n < 0 || n > INT_MAX)
        return sr_fail(ctx, SR_EINVAL, "n out of range");
    if (n > 0 && (!vx || !vy || !vz))
        return sr_fail(ctx, SR_EINVAL, "NULL velocity pointer with n > 0");
    if (!std::isfinite(dt))
        return sr_fail(ctx, SR_EINVAL, "dt must be finite");
    SplitGeom sg;
    int rc = split_geom(ctx, box, cell, &sg);
    if (rc)
        return rc;
    // validates the remaining arguments before anything is enqueued
    size_t bytes = 0;
    if ((rc = force_split_masked(ctx, cell3, ox, oy, oz, mass, n, box, cell, r_max, eps, poly, ax,
                                 ay, az, nullptr, nullptr, &bytes)))
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    const int ni = (int)n;
    // the serving maps: stream by dt/2 in FP64, kick by fl32(dt)
    const double half = 0.5 * (double)dt;
    if ((rc = kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, nullptr, nullptr,
                                  nullptr, 0.f, half)))
        return rc;
    if ((rc = force_split_masked(ctx, cell3, ox, oy, oz, mass, n, box, cell, r_max, eps, poly, ax,
                                 ay, az, nullptr, nullptr, nullptr)))
        return rc;
    return kick_stream_enqueue(ctx, sg, ni, cell3, ox, oy, oz, vx, vy, vz, ax, ay, az, dt, half);
}
