// Context, scratch arena, geometry validation and error reporting of libsr.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "sr_internal.h"

int sr_fail(sr_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int sr_check_launch(sr_ctx *ctx, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return SR_OK;
}

extern "C" int sr_grid_dims(const sr_box *box, double cell, int32_t dims[3], int64_t *n_cells)
{
    if (!box || !dims || !(cell > 0.0) || !std::isfinite(cell))
        return SR_EINVAL;
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        double L = box->len[d];
        if (!(L > 0.0) || !std::isfinite(L))
            return SR_EINVAL;
        double q = std::floor(L / cell);
        if (q < 1.0 || q > 2147483647.0)
            return SR_EINVAL;
        dims[d] = (int32_t)q;
        total *= dims[d];
        if (total > 2147483646LL)
            return SR_EINVAL;
    }
    if (n_cells)
        *n_cells = total;
    return SR_OK;
}

int sr_make_geom(sr_ctx *ctx, const sr_box *box, double cell, Geom *g, int xsplit)
{
    int32_t dims[3];
    int64_t nc = 0;
    if (!box)
        return sr_fail(ctx, SR_EINVAL, "box is NULL");
    if (sr_grid_dims(box, cell, dims, &nc) != SR_OK)
        return sr_fail(ctx, SR_EINVAL, "bad geometry: len=(%g,%g,%g) cell=%g", box->len[0],
                       box->len[1], box->len[2], cell);
    if (xsplit < 1 || xsplit > kMaxXsplit)
        return sr_fail(ctx, SR_EINVAL, "xsplit %d out of [1, %d]", xsplit, kMaxXsplit);
    if ((int64_t)dims[0] * xsplit * dims[1] * dims[2] > 2147483646LL)
        return sr_fail(ctx, SR_EINVAL, "too many cells");
    dims[0] *= xsplit;
    nc *= xsplit;
    g->hx = xsplit;
    for (int d = 0; d < 3; ++d) {
        g->len[d] = box->len[d];
        g->inv[d] = (double)dims[d] / box->len[d];
        g->lenf[d] = (float)box->len[d];
        g->nc[d] = dims[d];
        g->w[d] = box->len[d] / (double)dims[d];
        // the pair loop pads tiles with sources at 1e6 on every axis (kFar,
        // sr_pair.h): a bounded side keeps them beyond every cutoff from
        // every real particle
        if (box->len[d] > kMaxSide)
            return sr_fail(ctx, SR_EINVAL, "box side %g exceeds %g", box->len[d], kMaxSide);
        if ((double)g->lenf[d] != box->len[d])
            return sr_fail(ctx, SR_EINVAL, "box side %g is not exactly representable in float32",
                           box->len[d]);
    }
    g->ncell = (int)nc;
    div_const((unsigned)(g->nc[0] * g->nc[1]), &g->div_m[0], &g->div_s[0]);
    div_const((unsigned)g->nc[0], &g->div_m[1], &g->div_s[1]);
    g->split = 0;
    g->periodic = box->periodic ? 1 : 0;
    g->skin = box->periodic ? 0.0 : box->skin;
    if (!box->periodic && !(box->skin >= 0.0))
        return sr_fail(ctx, SR_EINVAL, "skin must be >= 0");
    return SR_OK;
}

int sr_arena_reserve(sr_ctx *ctx, size_t need)
{
    if (need > ctx->high_water)
        ctx->high_water = need;
    if (need <= ctx->arena_cap)
        return SR_OK;
    if (ctx->fixed)
        return sr_fail(ctx, SR_ENOMEM, "scratch arena of %zu bytes is too small: need %zu",
                       ctx->arena_cap, need);
    // grow: previous work may still read the old arena
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipStreamSynchronize failed while growing the arena");
    if (ctx->arena)
        (void)hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_cap = 0;
    size_t want = need + need / 4 + (1u << 20);
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return sr_fail(ctx, SR_ENOMEM, "hipMalloc(%zu) failed", want);
    }
    ctx->arena = (char *)p;
    ctx->arena_cap = want;
    return SR_OK;
}

extern "C" int sr_ctx_create(int device, void *hip_stream, size_t arena_bytes, sr_ctx **out)
{
    if (!out)
        return SR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return SR_EINVAL;
    if (hipSetDevice(device) != hipSuccess)
        return SR_EDEVICE;
    sr_ctx *ctx = new (std::nothrow) sr_ctx();
    if (!ctx)
        return SR_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    // device address of sr_force_static's fixed scratch on this device
    if (static_scratch_setup(device) != SR_OK) {
        delete ctx;
        return SR_EDEVICE;
    }
    void *p = nullptr;
    if (hipMalloc(&p, 256) != hipSuccess) {
        delete ctx;
        return SR_ENOMEM;
    }
    ctx->status = (int *)p;
    ctx->stats = (int64_t *)((char *)p + 64);
    if (hipMemset(p, 0, 256) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming) != hipSuccess) {
        if (ctx->handoff)
            (void)hipEventDestroy(ctx->handoff);
        (void)hipFree(p);
        delete ctx;
        return SR_EDEVICE;
    }
    if (arena_bytes > 0) {
        ctx->fixed = true;
        if (hipMalloc(&p, arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(ctx->status);
            (void)hipEventDestroy(ctx->handoff);
            delete ctx;
            return SR_ENOMEM;
        }
        ctx->arena = (char *)p;
        ctx->arena_cap = arena_bytes;
    }
    *out = ctx;
    return SR_OK;
}

extern "C" int sr_ctx_destroy(sr_ctx *ctx)
{
    if (!ctx)
        return SR_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->arena)
        (void)hipFree(ctx->arena);
    if (ctx->status)
        (void)hipFree(ctx->status);
    for (hipEvent_t e : ctx->events)
        (void)hipEventDestroy(e);
    if (ctx->handoff)
        (void)hipEventDestroy(ctx->handoff);
    delete ctx;
    return SR_OK;
}

int sr_timing_begin(sr_ctx *ctx)
{
    if (!ctx->timing)
        return -1;
    size_t need = ctx->events_used + 3;
    while (ctx->events.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return -1;
        ctx->events.push_back(e);
    }
    int rec = (int)(ctx->events_used / 3);
    ctx->events_used = need;
    return rec;
}

void sr_timing_mark(sr_ctx *ctx, int rec, int which)
{
    if (rec >= 0)
        (void)hipEventRecord(ctx->events[3 * (size_t)rec + which], ctx->stream);
}

extern "C" int sr_set_tuning(sr_ctx *ctx, const sr_tuning *t)
{
    if (!ctx || !t)
        return SR_EINVAL;
    if (t->xsplit < 1 || t->xsplit > kMaxXsplit)
        return sr_fail(ctx, SR_EINVAL, "xsplit must be in [1, %d]", kMaxXsplit);
    if (t->order < 0 || t->order > 1 || t->persistent < 0 || t->persistent > 1)
        return sr_fail(ctx, SR_EINVAL, "order and persistent must be 0 or 1");
    ctx->xsplit = t->xsplit;
    ctx->order = t->order;
    ctx->persistent = t->persistent;
    return SR_OK;
}

extern "C" int sr_get_tuning(const sr_ctx *ctx, sr_tuning *t)
{
    if (!ctx || !t)
        return SR_EINVAL;
    t->xsplit = ctx->xsplit;
    t->order = ctx->order;
    t->persistent = ctx->persistent;
    t->cell_scale = 1.0f;
    return SR_OK;
}

extern "C" int sr_timing_enable(sr_ctx *ctx, int enable)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->timing = enable != 0;
    return SR_OK;
}

extern "C" int sr_timing_collect(sr_ctx *ctx, double *prep_ms, double *force_ms, int64_t *calls)
{
    if (!ctx)
        return SR_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipStreamSynchronize failed");
    double p = 0.0, f = 0.0;
    size_t nrec = ctx->events_used / 3;
    for (size_t r = 0; r < nrec; ++r) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, ctx->events[3 * r], ctx->events[3 * r + 1]) != hipSuccess ||
            hipEventElapsedTime(&b, ctx->events[3 * r + 1], ctx->events[3 * r + 2]) != hipSuccess)
            return sr_fail(ctx, SR_EDEVICE, "hipEventElapsedTime failed");
        p += a;
        f += b;
    }
    ctx->events_used = 0;
    if (prep_ms)
        *prep_ms = p;
    if (force_ms)
        *force_ms = f;
    if (calls)
        *calls = (int64_t)nrec;
    return SR_OK;
}

extern "C" const char *sr_last_error(const sr_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "context is NULL";
}

// Every call shares the context's scratch arena, status word and counters,
// so work enqueued on a new stream must not start before the work already
// queued on the old one: the new stream waits for an event recorded on the
// old one (no host wait).
extern "C" int sr_set_stream(sr_ctx *ctx, void *hip_stream)
{
    if (!ctx)
        return SR_EINVAL;
    const hipStream_t next = (hipStream_t)hip_stream;
    if (next == ctx->stream)
        return SR_OK;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipEventRecord(ctx->handoff, ctx->stream) != hipSuccess ||
        hipStreamWaitEvent(next, ctx->handoff, 0) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "ordering the new stream after the old one failed");
    ctx->stream = next;
    return SR_OK;
}

extern "C" int sr_arena_info(const sr_ctx *ctx, size_t *allocated, size_t *high_water)
{
    if (!ctx)
        return SR_EINVAL;
    if (allocated)
        *allocated = ctx->arena_cap;
    if (high_water)
        *high_water = ctx->high_water;
    return SR_OK;
}

extern "C" int sr_sync(sr_ctx *ctx)
{
    if (!ctx)
        return SR_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipStreamSynchronize: %s",
                       hipGetErrorString(hipGetLastError()));
    int st = 0;
    if (hipMemcpy(&st, ctx->status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "reading the status word failed");
    if (st != 0) {
        int zero = 0;
        (void)hipMemcpy(ctx->status, &zero, sizeof(int), hipMemcpyHostToDevice);
        if (st & 2)
            return sr_fail(ctx, SR_ERANGE, "a mass was negative or not finite, or a PM position "
                                           "was not finite");
        return sr_fail(ctx, SR_ERANGE, "a coordinate was outside [0, L) or NaN");
    }
    return SR_OK;
}
