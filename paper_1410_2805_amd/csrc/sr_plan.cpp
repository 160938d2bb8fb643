// Batched form: a plan holds many independent boxes, their device
// descriptor table and scratch, and replays one pass (binning, work items,
// pair loop, per-box FP64 momentum) directly or as a captured HIP graph.
// It also carries the project's autotuner over the pair-loop tiling.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "sr_internal.h"

struct sr_plan {
    sr_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<sr_batch_box> boxes;
    float r_max = 0.f;
    ForceParams fp{};
    double *momentum = nullptr;
    sr_tuning tuning{2, 1, 0, 1.0f};
    // device memory: descriptor table, starts, scratch
    char *mem = nullptr;
    BoxDesc *d_boxes = nullptr;
    int *d_pstart = nullptr;
    int *d_cstart = nullptr;
    ForceScratch s{};
    int ntot = 0;
    int ctot = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// Runs f with the context's stream switched to the plan's stream.
template <class F>
int on_plan_stream(sr_plan *p, F f)
{
    hipStream_t saved = p->ctx->stream;
    p->ctx->stream = p->stream;
    int rc = f();
    p->ctx->stream = saved;
    return rc;
}

void drop_graph(sr_plan *p)
{
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// x sub-cells of box bx under tuning t: split-coordinate boxes take at most
// 3 (their stencil has one piece per cell, 9 (2 xsplit + 1) <= 63).
int box_xsplit(const sr_batch_box &bx, const sr_tuning &t)
{
    return bx.cell3 && t.xsplit > 3 ? 3 : t.xsplit;
}

// Geometry of every box under a tuning; returns SR_EINVAL naming the box.
int box_geoms(sr_plan *p, const sr_tuning &t, std::vector<Geom> &g, int64_t *ctot)
{
    g.resize(p->boxes.size());
    int64_t c = 0;
    for (size_t b = 0; b < p->boxes.size(); ++b) {
        const sr_batch_box &bx = p->boxes[b];
        const int xs = box_xsplit(bx, t);
        int rc = check_box_args(p->ctx, &bx.box, bx.cell * (double)t.cell_scale, p->r_max, xs,
                                &g[b]);
        if (rc)
            return sr_fail(p->ctx, rc, "box %zu: %s", b, p->ctx->err.c_str());
        if (bx.cell3) {
            // the offsets are relative to the mesh of `cell`: no other mesh
            if (t.cell_scale != 1.0f)
                return sr_fail(p->ctx, SR_EINVAL, "box %zu: split coordinates need cell_scale 1",
                               b);
            if (!bx.box.periodic)
                return sr_fail(p->ctx, SR_EINVAL, "box %zu: split coordinates need a periodic box",
                               b);
            for (int d = 0; d < 3; ++d)
                if (g[b].nc[d] / (d == 0 ? xs : 1) > kSplitMaxCells)
                    return sr_fail(p->ctx, SR_EINVAL,
                                   "box %zu: split coordinates allow at most %d cells per axis", b,
                                   kSplitMaxCells);
            g[b].split = 1;
        }
        c += g[b].ncell;
        if (c > 2147483646LL)
            return sr_fail(p->ctx, SR_EINVAL, "too many cells in the batch");
    }
    *ctot = c;
    return SR_OK;
}

// Upload the descriptor table for a tuning (waits for the copy).
int configure(sr_plan *p, const sr_tuning &t)
{
    if (t.xsplit < 1 || t.xsplit > kMaxXsplit || t.order < 0 || t.order > 1 ||
        t.persistent < 0 || t.persistent > 1 || !(t.cell_scale >= 1.0f) ||
        !std::isfinite(t.cell_scale))
        return sr_fail(p->ctx, SR_EINVAL, "invalid tuning");
    std::vector<Geom> g;
    int64_t ctot = 0;
    int rc = box_geoms(p, t, g, &ctot);
    if (rc)
        return rc;
    const int nb = (int)p->boxes.size();
    std::vector<BoxDesc> d(nb);
    std::vector<int> ps(nb + 1), cs(nb + 1);
    int pb = 0, cb = 0;
    for (int b = 0; b < nb; ++b) {
        const sr_batch_box &bx = p->boxes[b];
        d[b] = BoxDesc{};
        d[b].g = g[b];
        d[b].pbase = pb;
        d[b].n = (int)bx.n;
        d[b].cbase = cb;
        d[b].x = bx.x;
        d[b].y = bx.y;
        d[b].z = bx.z;
        d[b].m = bx.mass;
        d[b].cell3 = bx.cell3;
        d[b].ax = bx.ax;
        d[b].ay = bx.ay;
        d[b].az = bx.az;
        ps[b] = pb;
        cs[b] = cb;
        pb += (int)bx.n;
        cb += g[b].ncell;
    }
    ps[nb] = pb;
    cs[nb] = cb;
    if (hipStreamSynchronize(p->stream) != hipSuccess ||
        hipMemcpy(p->d_boxes, d.data(), sizeof(BoxDesc) * nb, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_pstart, ps.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_cstart, cs.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice) !=
            hipSuccess)
        return sr_fail(p->ctx, SR_EDEVICE, "uploading the box table failed");
    drop_graph(p);
    p->ctot = (int)ctot;
    p->tuning = t;
    return SR_OK;
}

Batch batch_of(const sr_plan *p)
{
    Batch B{};
    B.boxes = p->d_boxes;
    B.pstart = p->d_pstart;
    B.cstart = p->d_cstart;
    B.nb = (int)p->boxes.size();
    B.ntot = p->ntot;
    B.ctot = p->ctot;
    return B;
}

int enqueue(sr_plan *p)
{
    const Batch B = batch_of(p);
    return on_plan_stream(p, [&] {
        return force_enqueue(p->ctx, B, p->s, p->fp, p->tuning.order, p->tuning.persistent,
                             p->momentum, -1);
    });
}

}  // namespace

extern "C" int sr_plan_create(sr_ctx *ctx, const sr_batch_box *boxes, int nboxes, float r_max,
                              float eps, const float poly[6], double *momentum, sr_plan **out)
{
    if (!ctx || !out)
        return SR_EINVAL;
    *out = nullptr;
    ctx->err.clear();
    if (nboxes < 1 || !boxes)
        return sr_fail(ctx, SR_EINVAL, "need at least one box");
    if (nboxes > kMaxBatchBoxes)
        return sr_fail(ctx, SR_EINVAL, "at most %d boxes per plan", kMaxBatchBoxes);
    int rc = check_force_params(ctx, r_max, eps, poly);
    if (rc)
        return rc;
    int64_t ntot = 0;
    bool split_ok = false;  // some box may cut its chunks into sub-items
    for (int b = 0; b < nboxes; ++b) {
        const sr_batch_box &bx = boxes[b];
        if (bx.n < 0 || (bx.n > 0 && (!bx.x || !bx.y || !bx.z || !bx.mass || !bx.ax ||
                                      !bx.ay || !bx.az)))
            return sr_fail(ctx, SR_EINVAL, "box %d: bad size or NULL pointer", b);
        ntot += bx.n;
        split_ok = split_ok || box_splits(bx.n);
    }
    if (ntot > 2147483647LL)
        return sr_fail(ctx, SR_EINVAL, "too many particles in the batch");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    sr_plan *p = new (std::nothrow) sr_plan();
    if (!p)
        return SR_ENOMEM;
    p->ctx = ctx;
    p->boxes.assign(boxes, boxes + nboxes);
    p->r_max = r_max;
    p->fp = make_params(r_max, eps, poly);
    p->momentum = momentum;
    p->ntot = (int)ntot;
    p->tuning = sr_tuning{ctx->xsplit, ctx->order, ctx->persistent, 1.0f};
    if (ctx->stream) {
        p->stream = ctx->stream;
    } else {
        if (hipStreamCreate(&p->stream) != hipSuccess) {
            delete p;
            return sr_fail(ctx, SR_EDEVICE, "hipStreamCreate failed");
        }
        p->own_stream = true;
    }
    // scratch for the finest mesh any tuning can ask for (xsplit 4, scale 1)
    std::vector<Geom> g;
    int64_t ctot_max = 0;
    sr_tuning finest{kMaxXsplit, 1, 0, 1.0f};
    if ((rc = box_geoms(p, finest, g, &ctot_max))) {
        sr_plan_destroy(p);
        return rc;
    }
    Bump sz{nullptr, 0, 0};
    sz.take<BoxDesc>(nboxes);
    sz.take<int>(nboxes + 1);
    sz.take<int>(nboxes + 1);
    ForceScratch tmp;
    force_layout(sz, ntot, ctot_max, nboxes, tmp, false, split_ok);
    void *mem = nullptr;
    if (hipMalloc(&mem, sz.off) != hipSuccess) {
        (void)hipGetLastError();
        sr_plan_destroy(p);
        return sr_fail(ctx, SR_ENOMEM, "hipMalloc(%zu) for the plan failed", sz.off);
    }
    p->mem = (char *)mem;
    Bump b{p->mem, 0, sz.off};
    p->d_boxes = b.take<BoxDesc>(nboxes);
    p->d_pstart = b.take<int>(nboxes + 1);
    p->d_cstart = b.take<int>(nboxes + 1);
    force_layout(b, ntot, ctot_max, nboxes, p->s, false, split_ok);
    if ((rc = configure(p, p->tuning))) {
        sr_plan_destroy(p);
        return rc;
    }
    *out = p;
    return SR_OK;
}

extern "C" int sr_plan_set_tuning(sr_plan *plan, const sr_tuning *t)
{
    if (!plan || !t)
        return SR_EINVAL;
    return configure(plan, *t);
}

extern "C" int sr_plan_get_tuning(const sr_plan *plan, sr_tuning *t)
{
    if (!plan || !t)
        return SR_EINVAL;
    *t = plan->tuning;
    return SR_OK;
}

extern "C" int sr_plan_run(sr_plan *plan)
{
    if (!plan)
        return SR_EINVAL;
    plan->ctx->err.clear();
    return enqueue(plan);
}

extern "C" int sr_plan_capture(sr_plan *plan)
{
    if (!plan)
        return SR_EINVAL;
    drop_graph(plan);
    if (hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return sr_fail(plan->ctx, SR_EDEVICE, "hipStreamBeginCapture failed");
    int rc = enqueue(plan);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(plan->stream, &g);
    if (rc || e != hipSuccess || !g) {
        if (g)
            (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc ? rc : sr_fail(plan->ctx, SR_EDEVICE, "hipStreamEndCapture failed");
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return sr_fail(plan->ctx, SR_EDEVICE, "hipGraphInstantiate failed");
    }
    plan->graph = g;
    plan->exec = x;
    return SR_OK;
}

extern "C" int sr_plan_launch(sr_plan *plan)
{
    if (!plan)
        return SR_EINVAL;
    if (!plan->exec) {
        int rc = sr_plan_capture(plan);
        if (rc)
            return rc;
    }
    if (hipGraphLaunch(plan->exec, plan->stream) != hipSuccess)
        return sr_fail(plan->ctx, SR_EDEVICE, "hipGraphLaunch failed");
    return SR_OK;
}

extern "C" int sr_plan_autotune(sr_plan *plan, int reps, sr_tuning *best, double *best_ms)
{
    if (!plan || reps < 1)
        return SR_EINVAL;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return sr_fail(plan->ctx, SR_EDEVICE, "hipEventCreate failed");
    const sr_tuning start = plan->tuning;
    sr_tuning win = start;
    double win_ms = 1e300;
    int rc = SR_OK;
    const float scales[2] = {1.0f, 1.25f};
    for (float sc : scales)
        for (int xs = 1; xs <= 3; ++xs)
            for (int ord = 0; ord <= 1; ++ord)
                for (int per = 0; per <= 1; ++per) {
                    sr_tuning t{xs, ord, per, sc};
                    if (configure(plan, t) != SR_OK) {
                        plan->ctx->err.clear();
                        continue;  // e.g. a box too small for this cell scale
                    }
                    std::vector<double> ms;
                    if ((rc = enqueue(plan)))
                        goto done;
                    for (int r = 0; r < reps; ++r) {
                        (void)hipEventRecord(e0, plan->stream);
                        if ((rc = enqueue(plan)))
                            goto done;
                        (void)hipEventRecord(e1, plan->stream);
                        if (hipEventSynchronize(e1) != hipSuccess) {
                            rc = sr_fail(plan->ctx, SR_EDEVICE, "hipEventSynchronize failed");
                            goto done;
                        }
                        float f = 0.f;
                        (void)hipEventElapsedTime(&f, e0, e1);
                        ms.push_back(f);
                    }
                    std::sort(ms.begin(), ms.end());
                    const double med = ms[ms.size() / 2];
                    if (med < win_ms) {
                        win_ms = med;
                        win = t;
                    }
                }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        (void)configure(plan, start);
        return rc;
    }
    if ((rc = configure(plan, win)))
        return rc;
    if (best)
        *best = win;
    if (best_ms)
        *best_ms = win_ms;
    return SR_OK;
}

extern "C" int sr_plan_destroy(sr_plan *plan)
{
    if (!plan)
        return SR_EINVAL;
    if (plan->stream)
        (void)hipStreamSynchronize(plan->stream);
    drop_graph(plan);
    if (plan->mem)
        (void)hipFree(plan->mem);
    if (plan->own_stream)
        (void)hipStreamDestroy(plan->stream);
    delete plan;
    return SR_OK;
}
