// The batched scan for callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation): the
// partial answers live in a fixed, file-scope device array instead of a
// library-allocated per-stream workspace.
//
// `scratch` is a host-side stand-in in host code: its device address, which
// differs per GPU, is looked up once per device with hipGetSymbolAddress
// when a context is created on it (with that device current) and kept; only
// that address is ever passed to kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "pir_internal.h"
#include "pir_runtime.h"

namespace pir {

namespace {

static __device__ __align__(256) uint8_t scratch[PIR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

}  // namespace

int noalloc_scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PIR_E_DEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PIR_OK;
}

}  // namespace pir

using namespace pir;

extern "C" int pir_dpxor_batch_async_noalloc(pir_db* d, const void* d_sel, uint64_t sel_stride, uint32_t q,
                                             void* d_out, void* hip_stream) {
    clear_error();
    Db* db = reinterpret_cast<Db*>(d);
    int rc = check_async_args(db, d_sel, sel_stride, q, d_out);
    if (rc) return rc;
    Ctx* ctx = db->ctx;
    rc = ctx->bind();
    if (rc) return rc;
    if (!ctx->noalloc_scratch) return fail(PIR_E_DEVICE, "no fixed scratch on device %d", ctx->device);
    Plan p;
    rc = ctx->plan_for(*db, q, nullptr, p);
    if (rc) return rc;
    // the partials of every record group must fit the fixed scratch: fewer,
    // longer record groups where they would not (the answers do not depend
    // on the grouping); an error where even the fewest groups the exact
    // matrix-core counts allow do not fit
    const uint64_t per_group = (uint64_t)q * db->geo.rpad;
    if (partial_bytes(db->geo, p, q) > PIR_NOALLOC_SCRATCH_BYTES) {
        p.groups = (uint32_t)std::max<uint64_t>(1, PIR_NOALLOC_SCRATCH_BYTES / per_group);
        p.units_per_group = 0;
        rc = finish_plan(db->geo, q, p);
        if (rc) return rc;
        if (partial_bytes(db->geo, p, q) > PIR_NOALLOC_SCRATCH_BYTES)
            return fail(PIR_E_INVAL,
                        "pir_dpxor_batch_async_noalloc: %u queries x %u-byte records need %llu bytes of partial "
                        "answers, more than the %u-byte fixed scratch",
                        q, db->geo.R, (unsigned long long)partial_bytes(db->geo, p, q), (unsigned)PIR_NOALLOC_SCRATCH_BYTES);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    uint8_t* partials = (uint8_t*)ctx->noalloc_scratch;
    hipError_t he;
    if (p.variant == PIR_VARIANT_VALU)
        he = launch_stage1_valu(db->geo, p, db->data.ptr, (const uint32_t*)d_sel, sel_stride / 4, q, partials, s);
    else
        he = launch_stage1_mfma(db->geo, p, db->data.ptr, (const uint32_t*)d_sel, sel_stride / 4, q, partials, s);
    if (he != hipSuccess) return hip_fail(he, "stage-1 launch");
    he = launch_stage2(db->geo, p.groups, q, partials, (uint8_t*)d_out, s);
    if (he != hipSuccess) return hip_fail(he, "stage-2 launch");
    return PIR_OK;
}
