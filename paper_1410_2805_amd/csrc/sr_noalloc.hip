// sr_force with its scratch in a fixed device array instead of the context
// arena, for callers that cannot allocate device memory while they run
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Same kernels, same arithmetic: results are bitwise those of
// sr_force at the same tuning.
//
// The array is one per GPU, held from the library's load until the process
// ends.  Host code never passes its name to a kernel: the name is a host
// stand-in, not a device address.  Its device address is looked up once per
// device (with that device current) when a context is created there, and
// only that address is used afterwards.
#include <climits>
#include <mutex>

#include "sr_internal.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of scratch on each device, once looked up

}  // namespace

// Called by sr_ctx_create with `device` current.
int static_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return SR_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device])
        return SR_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return SR_EDEVICE;
    }
    g_ptr[device] = ptr;
    return SR_OK;
}

extern "C" size_t sr_force_static_capacity(void) { return kStaticScratchBytes; }

extern "C" int sr_force_static(sr_ctx *ctx, const float *x, const float *y, const float *z,
                               const float *mass, int64_t n, const sr_box *box, double cell,
                               float r_max, float eps, const float poly[6], float *ax, float *ay,
                               float *az, double *momentum3)
{
    if (!ctx)
        return SR_EINVAL;
    ctx->err.clear();
    int rc = check_force_params(ctx, r_max, eps, poly);
    if (rc)
        return rc;
    Batch B;
    if ((rc = single_batch(ctx, x, y, z, mass, n, box, cell, r_max, ctx->xsplit, ax, ay, az, &B)))
        return rc;
    if (n > 0 && (!mass || !ax || !ay || !az))
        return sr_fail(ctx, SR_EINVAL, "NULL mass or output pointer");
    Bump sz{nullptr, 0, 0};
    ForceScratch s;
    force_layout(sz, n, B.ctot, 1, s, false, box_splits(n));
    if (sz.off > kStaticScratchBytes)
        return sr_fail(ctx, SR_ENOMEM,
                       "sr_force_static: %zu scratch bytes needed, the fixed array holds %zu "
                       "(n=%lld, %d cells)",
                       sz.off, kStaticScratchBytes, (long long)n, B.ctot);
    void *ptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ptr = ctx->device < kMaxDevices ? g_ptr[ctx->device] : nullptr;
    }
    if (!ptr)
        return sr_fail(ctx, SR_EDEVICE, "sr_force_static: no device address for the scratch array");
    if (hipSetDevice(ctx->device) != hipSuccess)
        return sr_fail(ctx, SR_EDEVICE, "hipSetDevice failed");
    Bump b{(char *)ptr, 0, kStaticScratchBytes};
    force_layout(b, n, B.ctot, 1, s, false, box_splits(n));
    const ForceParams fp = make_params(r_max, eps, poly);
    // no timing record: its events would be created on demand
    return force_enqueue(ctx, B, s, fp, ctx->order, ctx->persistent, momentum3, -1);
}
