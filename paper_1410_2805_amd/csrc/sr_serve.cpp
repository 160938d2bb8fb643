// Serving form: continuous batching of stream-kick-stream requests.
//
// Requests queue in arrival order and are admitted while a slot, state
// memory (a first-fit pool carved from one HBM allocation, in the spirit of
// the Bigchunk allocator of Sec. 2.7) and pass scratch allow.  Every tick
// advances all admitted requests by one step with one batched pass: stream
// half step, segmented binning, one pair-loop launch over every request's
// work items, kick and stream half step.  State is resident in split
// coordinates (cell + float32 offset) from admission until the request's
// last step, when its float64 positions and velocities are copied back and
// an event marks completion.  Requests that arrive while others run join at
// the next tick; each request's arithmetic is independent of the mix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "sr_internal.h"
#include "sr_split.h"

namespace {

constexpr int kRing = 4;  // descriptor buffers in flight

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// First-fit allocator with coalescing over [0, cap).
struct Pool {
    size_t cap = 0, used = 0, high = 0;
    std::map<size_t, size_t> free_;
    void init(size_t c)
    {
        cap = c;
        used = high = 0;
        free_.clear();
        if (c)
            free_[0] = c;
    }
    bool alloc(size_t len, size_t *off)
    {
        len = al(len);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len)
                continue;
            *off = it->first;
            const size_t rem = it->second - len, o2 = it->first + len;
            free_.erase(it);
            if (rem)
                free_[o2] = rem;
            used += len;
            high = std::max(high, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t len)
    {
        len = al(len);
        used -= len;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

enum { kQueued = 0, kActive = 1, kDraining = 2, kCancelled = 3 };

struct Req {
    sr_request r{};
    int state = kQueued;
    size_t off = 0, bytes = 0;
    int steps_done = 0;
    SplitGeom sg{};
    Geom g{};
    int *cell3 = nullptr;
    float *ox = nullptr, *oy = nullptr, *oz = nullptr;
    float *vx = nullptr, *vy = nullptr, *vz = nullptr;
    float *m = nullptr, *ax = nullptr, *ay = nullptr, *az = nullptr;
    double *fx = nullptr, *fy = nullptr, *fz = nullptr;
    double *kin = nullptr;  // kRedBlocks partials, then K
    hipEvent_t done = nullptr;
};

size_t state_bytes(int64_t n)
{
    const size_t f = al((size_t)n * 4), d = al((size_t)n * 8);
    return f /*cell3*/ + 3 * f /*o*/ + 3 * f /*v*/ + f /*m*/ + 3 * f /*a*/ + 3 * d /*f64*/ +
           al((kRedBlocks + 1) * sizeof(double)) /*K*/;
}

void carve(Req &q, char *base)
{
    const size_t f = al((size_t)q.r.n * 4), d = al((size_t)q.r.n * 8);
    char *p = base + q.off;
    q.cell3 = (int *)p;
    p += f;
    float **fl[10] = {&q.ox, &q.oy, &q.oz, &q.vx, &q.vy, &q.vz, &q.m, &q.ax, &q.ay, &q.az};
    for (float **x : fl) {
        *x = (float *)p;
        p += f;
    }
    q.fx = (double *)p;
    q.fy = (double *)(p + d);
    q.fz = (double *)(p + 2 * d);
    q.kin = (double *)(p + 3 * d);
}

size_t table_bytes(int slots)
{
    return al(sizeof(BoxDesc) * slots) + al(sizeof(SlotState) * slots) +
           2 * al(sizeof(int) * (slots + 1));
}

}  // namespace

struct sr_server {
    sr_ctx *ctx = nullptr;
    sr_server_config cfg{};
    ForceParams fp{};
    int xsplit = 1;
    char *pool_mem = nullptr;
    Pool pool;
    char *scratch = nullptr;
    size_t scratch_cap = 0;
    char *dev_tab[kRing] = {};
    char *host_tab[kRing] = {};
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    size_t tab_cap = 0;
    std::deque<int64_t> queue;
    std::map<int64_t, Req> reqs;
    std::vector<int64_t> active;
    std::vector<int64_t> finished;
    int64_t next_id = 1;
    int64_t ticks = 0;
    int64_t completed = 0;
};

namespace {

size_t scratch_need(const sr_server *S, int64_t ntot, int64_t ctot, int nb)
{
    Bump sz{nullptr, 0, 0};
    ForceScratch s;
    force_layout(sz, ntot, ctot, nb, s, false, true);  // any request may cut its chunks
    return sz.off;
}

void active_totals(const sr_server *S, int64_t *ntot, int64_t *ctot)
{
    *ntot = *ctot = 0;
    for (int64_t id : S->active) {
        const Req &q = S->reqs.at(id);
        *ntot += q.r.n;
        *ctot += q.g.ncell;
    }
}

int admit(sr_server *S)
{
    sr_ctx *ctx = S->ctx;
    while (!S->queue.empty() && (int)S->active.size() < S->cfg.max_slots) {
        const int64_t id = S->queue.front();
        Req &q = S->reqs.at(id);
        int64_t nt, ct;
        active_totals(S, &nt, &ct);
        if (nt + q.r.n > 2147483647LL ||
            scratch_need(S, nt + q.r.n, ct + q.g.ncell, (int)S->active.size() + 1) >
                S->scratch_cap)
            break;
        if (!S->pool.alloc(q.bytes, &q.off))
            break;
        carve(q, S->pool_mem);
        const size_t n = (size_t)q.r.n;
        if (hipMemcpyAsync(q.fx, q.r.x, n * 8, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.fy, q.r.y, n * 8, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.fz, q.r.z, n * 8, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.vx, q.r.vx, n * 4, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.vy, q.r.vy, n * 4, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.vz, q.r.vz, n * 4, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(q.m, q.r.mass, n * 4, hipMemcpyHostToDevice, ctx->stream) !=
                hipSuccess)
            return sr_fail(ctx, SR_EDEVICE, "admission copy failed");
        int rc = split_from_f64_enqueue(ctx, q.fx, q.fy, q.fz, (int)n, q.sg, q.cell3, q.ox, q.oy,
                                        q.oz);
        if (rc)
            return rc;
        q.state = kActive;
        q.steps_done = 0;
        S->active.push_back(id);
        S->queue.pop_front();
    }
    return SR_OK;
}

}  // namespace

extern "C" int sr_server_create(sr_ctx *ctx, const sr_server_config *cfg, sr_server **out)
{
    if (!ctx || !cfg || !out)
        return SR_EINVAL;
    *out = nullptr;
    ctx->err.clear();
    int rc = check_force_params(ctx, cfg->r_max, cfg->eps, cfg->poly);
    if (rc)
        return rc;
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxBatchBoxes ||
        cfg->hbm_budget < (size_t)(64u << 20) || !(cfg->cell > 0.0))
        return sr_fail(ctx, SR_EINVAL,
                       "need 1 <= max_slots <= %d, hbm_budget >= 64 MiB, cell > 0",
                       kMaxBatchBoxes);
    const sr_tuning &t = cfg->tuning;
    if (t.xsplit < 1 || t.xsplit > kMaxXsplit || t.order < 0 || t.order > 1 ||
        t.persistent < 0 || t.persistent > 1)
        return sr_fail(ctx, SR_EINVAL, "invalid tuning");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    sr_server *S = new (std::nothrow) sr_server();
    if (!S)
        return SR_ENOMEM;
    S->ctx = ctx;
    S->cfg = *cfg;
    S->fp = make_params(cfg->r_max, cfg->eps, cfg->poly);
    S->xsplit = t.xsplit < 3 ? t.xsplit : 3;
    const size_t half = al(cfg->hbm_budget / 2);
    S->tab_cap = table_bytes(cfg->max_slots);
    void *p = nullptr;
    if (hipMalloc(&p, half) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return sr_fail(ctx, SR_ENOMEM, "hipMalloc(%zu) for the state pool failed", half);
    }
    S->pool_mem = (char *)p;
    S->pool.init(half);
    if (hipMalloc(&p, half) != hipSuccess) {
        (void)hipGetLastError();
        sr_server_destroy(S);
        return sr_fail(ctx, SR_ENOMEM, "hipMalloc(%zu) for the scratch failed", half);
    }
    S->scratch = (char *)p;
    S->scratch_cap = half;
    for (int k = 0; k < kRing; ++k) {
        if (hipMalloc(&p, S->tab_cap) != hipSuccess) {
            sr_server_destroy(S);
            return sr_fail(ctx, SR_ENOMEM, "descriptor buffer allocation failed");
        }
        S->dev_tab[k] = (char *)p;
        if (hipHostMalloc(&p, S->tab_cap, hipHostMallocDefault) != hipSuccess) {
            sr_server_destroy(S);
            return sr_fail(ctx, SR_ENOMEM, "pinned descriptor buffer allocation failed");
        }
        S->host_tab[k] = (char *)p;
        if (hipEventCreateWithFlags(&S->ring_ev[k], hipEventDisableTiming) != hipSuccess) {
            sr_server_destroy(S);
            return sr_fail(ctx, SR_EDEVICE, "hipEventCreate failed");
        }
    }
    *out = S;
    return SR_OK;
}

extern "C" int sr_server_submit(sr_server *S, const sr_request *req, int64_t *id)
{
    if (!S || !req || !id)
        return SR_EINVAL;
    sr_ctx *ctx = S->ctx;
    ctx->err.clear();
    const sr_request &r = *req;
    if (r.n < 1 || r.n > 2147483647LL || r.steps < 1 || !std::isfinite(r.dt) || !r.x || !r.y ||
        !r.z || !r.vx || !r.vy || !r.vz || !r.mass || !r.out_x || !r.out_y || !r.out_z ||
        !r.out_vx || !r.out_vy || !r.out_vz)
        return sr_fail(ctx, SR_EINVAL, "invalid request (size, steps, dt or NULL pointer)");
    Req q;
    q.r = r;
    sr_box box{};
    box.len[0] = box.len[1] = box.len[2] = r.len;
    box.periodic = 1;
    int rc = check_box_args(ctx, &box, S->cfg.cell, S->cfg.r_max, S->xsplit, &q.g);
    if (rc)
        return rc;
    if ((rc = split_geom(ctx, &box, S->cfg.cell, &q.sg)))
        return rc;
    q.g.split = 1;
    q.bytes = state_bytes(r.n);
    if (al(q.bytes) > S->pool.cap || scratch_need(S, r.n, q.g.ncell, 1) > S->scratch_cap)
        return sr_fail(ctx, SR_EBUSY, "request of %lld particles can never fit the budget",
                       (long long)r.n);
    if (hipEventCreateWithFlags(&q.done, hipEventDisableTiming) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipEventCreate failed");
    const int64_t nid = S->next_id++;
    S->reqs.emplace(nid, q);
    S->queue.push_back(nid);
    *id = nid;
    return SR_OK;
}

extern "C" int sr_server_tick(sr_server *S, int *n_active)
{
    if (!S)
        return SR_EINVAL;
    sr_ctx *ctx = S->ctx;
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    int rc = admit(S);
    if (rc)
        return rc;
    const int nb = (int)S->active.size();
    if (n_active)
        *n_active = nb;
    if (nb == 0)
        return SR_OK;
    const int k = (int)(S->ticks % kRing);
    if (S->ring_used[k] && hipEventSynchronize(S->ring_ev[k]) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipEventSynchronize failed");
    // descriptor tables of this tick
    char *h = S->host_tab[k];
    BoxDesc *hb = (BoxDesc *)h;
    SlotState *hs = (SlotState *)(h + al(sizeof(BoxDesc) * S->cfg.max_slots));
    int *hp = (int *)((char *)hs + al(sizeof(SlotState) * S->cfg.max_slots));
    int *hc = (int *)((char *)hp + al(sizeof(int) * (S->cfg.max_slots + 1)));
    int pb = 0, cb = 0;
    for (int b = 0; b < nb; ++b) {
        Req &q = S->reqs.at(S->active[b]);
        BoxDesc d{};
        d.g = q.g;
        d.pbase = pb;
        d.n = (int)q.r.n;
        d.cbase = cb;
        d.x = q.ox;
        d.y = q.oy;
        d.z = q.oz;
        d.m = q.m;
        d.cell3 = q.cell3;
        d.ax = q.ax;
        d.ay = q.ay;
        d.az = q.az;
        hb[b] = d;
        SlotState st{};
        st.g = q.sg;
        st.dt = q.r.dt;
        st.cell3 = q.cell3;
        st.ox = q.ox;
        st.oy = q.oy;
        st.oz = q.oz;
        st.vx = q.vx;
        st.vy = q.vy;
        st.vz = q.vz;
        st.ax = q.ax;
        st.ay = q.ay;
        st.az = q.az;
        hs[b] = st;
        hp[b] = pb;
        hc[b] = cb;
        pb += d.n;
        cb += q.g.ncell;
    }
    hp[nb] = pb;
    hc[nb] = cb;
    char *dt = S->dev_tab[k];
    if (hipMemcpyAsync(dt, h, S->tab_cap, hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "descriptor upload failed");
    const BoxDesc *db = (const BoxDesc *)dt;
    const SlotState *ds = (const SlotState *)(dt + ((char *)hs - h));
    const int *dp = (const int *)(dt + ((char *)hp - h));
    const int *dc = (const int *)(dt + ((char *)hc - h));
    Batch B{};
    B.boxes = db;
    B.pstart = dp;
    B.cstart = dc;
    B.nb = nb;
    B.ntot = pb;
    B.ctot = cb;
    Bump bs{S->scratch, 0, S->scratch_cap};
    ForceScratch fs;
    force_layout(bs, pb, cb, nb, fs, false, true);
    if (bs.off > S->scratch_cap)
        return sr_fail(ctx, SR_ENOMEM, "scratch overflow (admission bug)");
    if ((rc = slot_update_enqueue(ctx, ds, dp, nb, pb, 0)))
        return rc;
    if ((rc = force_enqueue(ctx, B, fs, S->fp, S->cfg.tuning.order, S->cfg.tuning.persistent,
                            nullptr, -1)))
        return rc;
    if ((rc = slot_update_enqueue(ctx, ds, dp, nb, pb, 1)))
        return rc;
    if (hipEventRecord(S->ring_ev[k], ctx->stream) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipEventRecord failed");
    S->ring_used[k] = true;
    // retire finished requests: results to the host, completion event
    std::vector<int64_t> still;
    for (int64_t id : S->active) {
        Req &q = S->reqs.at(id);
        q.steps_done += 1;
        if (q.steps_done < q.r.steps) {
            still.push_back(id);
            continue;
        }
        const size_t n = (size_t)q.r.n;
        if ((rc = split_to_f64_enqueue(ctx, q.cell3, q.ox, q.oy, q.oz, (int)n, q.sg, q.fx, q.fy,
                                       q.fz)))
            return rc;
        if (hipMemcpyAsync(q.r.out_x, q.fx, n * 8, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess ||
            hipMemcpyAsync(q.r.out_y, q.fy, n * 8, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess ||
            hipMemcpyAsync(q.r.out_z, q.fz, n * 8, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess ||
            hipMemcpyAsync(q.r.out_vx, q.vx, n * 4, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess ||
            hipMemcpyAsync(q.r.out_vy, q.vy, n * 4, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess ||
            hipMemcpyAsync(q.r.out_vz, q.vz, n * 4, hipMemcpyDeviceToHost, ctx->stream) !=
                hipSuccess)
            return sr_fail(ctx, SR_EDEVICE, "result copy failed");
        if (q.r.out_kinetic) {
            if ((rc = kinetic_enqueue(ctx, q.vx, q.vy, q.vz, q.m, (int)n, q.kin,
                                      q.kin + kRedBlocks)))
                return rc;
            if (hipMemcpyAsync(q.r.out_kinetic, q.kin + kRedBlocks, sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
                return sr_fail(ctx, SR_EDEVICE, "result copy failed");
        }
        if (hipEventRecord(q.done, ctx->stream) != hipSuccess)
            return sr_fail(ctx, SR_EDEVICE, "hipEventRecord failed");
        q.state = kDraining;
    }
    S->active.swap(still);
    S->ticks += 1;
    return SR_OK;
}

extern "C" int sr_server_poll(sr_server *S, int64_t *ids, int cap, int *n)
{
    if (!S || !n || (cap > 0 && !ids))
        return SR_EINVAL;
    *n = 0;
    for (auto it = S->reqs.begin(); it != S->reqs.end();) {
        Req &q = it->second;
        if ((q.state == kDraining || q.state == kCancelled) &&
            hipEventQuery(q.done) == hipSuccess) {
            S->pool.release(q.off, q.bytes);
            if (q.state == kDraining) {
                S->finished.push_back(it->first);
                S->completed += 1;
            }
            (void)hipEventDestroy(q.done);
            it = S->reqs.erase(it);
        } else {
            ++it;
        }
    }
    int k = 0;
    while (k < cap && !S->finished.empty()) {
        ids[k++] = S->finished.front();
        S->finished.erase(S->finished.begin());
    }
    *n = k;
    return SR_OK;
}

extern "C" int sr_server_cancel(sr_server *S, int64_t id)
{
    if (!S)
        return SR_EINVAL;
    auto it = S->reqs.find(id);
    if (it == S->reqs.end())
        return sr_fail(S->ctx, SR_EINVAL, "unknown request %lld", (long long)id);
    Req &q = it->second;
    if (q.state == kQueued) {
        S->queue.erase(std::find(S->queue.begin(), S->queue.end(), id));
        (void)hipEventDestroy(q.done);
        S->reqs.erase(it);
        return SR_OK;
    }
    if (q.state == kActive) {
        S->active.erase(std::find(S->active.begin(), S->active.end(), id));
        // free once every pass enqueued so far is done with its memory
        if (hipEventRecord(q.done, S->ctx->stream) != hipSuccess)
            return sr_fail(S->ctx, SR_EDEVICE, "hipEventRecord failed");
        q.state = kCancelled;
        return SR_OK;
    }
    return sr_fail(S->ctx, SR_EINVAL, "request %lld already finished", (long long)id);
}

extern "C" int sr_server_info_get(const sr_server *S, sr_server_info *info)
{
    if (!S || !info)
        return SR_EINVAL;
    sr_server_info r{};
    for (const auto &kv : S->reqs) {
        if (kv.second.state == kQueued)
            r.queued++;
        else if (kv.second.state == kActive)
            r.active++;
        else if (kv.second.state == kDraining)
            r.draining++;
    }
    r.completed = S->completed;
    r.state_bytes_in_use = S->pool.used;
    r.state_bytes_high_water = S->pool.high;
    r.state_bytes_capacity = S->pool.cap;
    r.scratch_bytes_capacity = S->scratch_cap;
    r.ticks = S->ticks;
    *info = r;
    return SR_OK;
}

extern "C" int sr_server_destroy(sr_server *S)
{
    if (!S)
        return SR_EINVAL;
    (void)hipStreamSynchronize(S->ctx->stream);
    for (auto &kv : S->reqs)
        if (kv.second.done)
            (void)hipEventDestroy(kv.second.done);
    for (int k = 0; k < kRing; ++k) {
        if (S->dev_tab[k])
            (void)hipFree(S->dev_tab[k]);
        if (S->host_tab[k])
            (void)hipHostFree(S->host_tab[k]);
        if (S->ring_ev[k])
            (void)hipEventDestroy(S->ring_ev[k]);
    }
    if (S->pool_mem)
        (void)hipFree(S->pool_mem);
    if (S->scratch)
        (void)hipFree(S->scratch);
    delete S;
    return SR_OK;
}
