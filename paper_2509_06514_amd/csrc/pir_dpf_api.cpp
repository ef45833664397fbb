// C ABI of the DPF calls: client-side key generation (host), full-domain
// evaluation on the device, and the key-to-answer path that feeds the
// evaluated selection rows to the batched scan (IM-PIR Sec. 3.1-3.3).
#include <cstring>

#include "pir_runtime.h"

namespace pir {
namespace {

// The last launch of the evaluation chain has one thread per 32 leaves and
// a launch dimension holds fewer than 2^32 work-items: 2^(n-5) <= 2^31.
constexpr uint32_t kMaxDomainBits = 36;
constexpr uint64_t kNodeScratchBudget = 3ull << 29;  // tree-level scratch per call (1.5 GiB)
constexpr uint64_t kSelScratchBudget = 2ull << 30;   // selection rows of the key-to-answer path

uint64_t words_for(uint64_t n_leaves) { return (n_leaves + 31) / 32; }

// Keys per group so the node scratch stays within budget (at least one key),
// balanced so the groups differ in size by at most one.
uint32_t keys_per_group(uint32_t n, uint64_t n_leaves, uint32_t n_keys) {
    const uint64_t per_key = 2 * dpf_scratch_nodes(n, n_leaves) * 16;
    if (per_key == 0) return n_keys;
    uint64_t g = kNodeScratchBudget / per_key;
    if (g < 1) g = 1;
    if (g >= n_keys) return n_keys;
    const uint64_t groups = (n_keys + g - 1) / g;
    return (uint32_t)((n_keys + groups - 1) / groups);
}

// Grow a per-stream buffer; waits for the stream first if it is in use.
int grow(DevBuf& b, size_t need, hipStream_t s, const char* what) {
    if (need <= b.bytes) return PIR_OK;
    if (b.ptr) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, what);
    }
    hipError_t e = b.ensure(need);
    if (e != hipSuccess) return hip_fail(e, what);
    return PIR_OK;
}

}  // namespace

uint64_t dpf_eval_scratch_bytes(uint32_t n, uint64_t n_leaves, uint32_t n_keys) {
    return (uint64_t)keys_per_group(n, n_leaves, n_keys) * 2 * dpf_scratch_nodes(n, n_leaves) * 16 + 16;
}

namespace {

// Evaluate n_keys keys into rows of d_sel, in groups bounded by the node
// scratch budget.  Caller holds no lock; ws belongs to stream s.
int eval_groups(Ctx* ctx, const uint8_t* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves, uint32_t* d_sel,
                uint64_t stride_words, hipStream_t s) {
    const uint32_t gk = keys_per_group(n, n_leaves, n_keys);
    const uint64_t nodes = dpf_scratch_nodes(n, n_leaves);
    DevBuf* nb;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        nb = &ctx->dpf_ws[s].nodes;
    }
    int rc = grow(*nb, (size_t)gk * 2 * nodes * 16 + 16, s, "DPF scratch");
    if (rc) return rc;
    const bool timed = ctx->timing_on.load();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        e0 = ctx->take_event();
        e1 = ctx->take_event();
    }
    if (e0) (void)hipEventRecord(e0, s);
    const uint64_t kb = dpf_key_bytes(n);
    for (uint32_t k0 = 0; k0 < n_keys; k0 += gk) {
        const uint32_t nk = n_keys - k0 < gk ? n_keys - k0 : gk;
        hipError_t e = launch_dpf_eval(ctx->device, d_keys + (uint64_t)k0 * kb, n, nk, n_leaves,
                                       d_sel + (uint64_t)k0 * stride_words, stride_words, nb->ptr, nodes, s);
        if (e != hipSuccess) return hip_fail(e, "DPF evaluation launch");
    }
    if (e1) (void)hipEventRecord(e1, s);
    if (timed && e0 && e1) ctx->add_timed(e0, e1, 3);
    return PIR_OK;
}

}  // namespace

int dpf_eval_into(Ctx* ctx, const uint8_t* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves, uint32_t* d_sel,
                  uint64_t stride_words, hipStream_t s) {
    return eval_groups(ctx, d_keys, n, n_keys, n_leaves, d_sel, stride_words, s);
}

}  // namespace pir

using namespace pir;

extern "C" {

uint64_t pir_dpf_key_bytes(uint32_t n) { return dpf_key_bytes(n); }

uint32_t pir_dpf_domain_bits(uint64_t n_records) {
    uint32_t n = 0;
    while (n < 64 && (1ull << n) < n_records) ++n;
    return n;
}

int pir_dpf_gen(uint64_t alpha, uint32_t n, const uint8_t* root0, const uint8_t* root1, uint8_t* key0,
                uint8_t* key1) {
    clear_error();
    if (!root0 || !root1 || !key0 || !key1) return fail(PIR_E_INVAL, "pir_dpf_gen: NULL argument");
    if (n > 62) return fail(PIR_E_INVAL, "pir_dpf_gen: n=%u > 62", n);
    if (alpha >> n) return fail(PIR_E_INVAL, "pir_dpf_gen: alpha outside [0, 2^%u)", n);
    dpf_gen_host(alpha, n, root0, root1, key0, key1);
    return PIR_OK;
}

int pir_reconstruct(const uint8_t* ans0, const uint8_t* ans1, uint64_t record_bytes, uint8_t* out) {
    clear_error();
    if (!ans0 || !ans1 || !out) return fail(PIR_E_INVAL, "pir_reconstruct: NULL argument");
    for (uint64_t i = 0; i < record_bytes; ++i) out[i] = ans0[i] ^ ans1[i];
    return PIR_OK;
}

int pir_dpf_eval_async(pir_ctx* c, const void* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves,
                       void* d_sel, uint64_t sel_stride, void* hip_stream) {
    clear_error();
    Ctx* ctx = reinterpret_cast<Ctx*>(c);
    if (!ctx || !d_keys || !d_sel) return fail(PIR_E_INVAL, "pir_dpf_eval_async: NULL argument");
    if (n > kMaxDomainBits) return fail(PIR_E_INVAL, "n=%u > %u", n, kMaxDomainBits);
    if (n_keys == 0 || n_keys > PIR_MAX_BATCH)
        return fail(PIR_E_INVAL, "n_keys=%u outside [1, %u]", n_keys, PIR_MAX_BATCH);
    if (n_leaves == 0 || n_leaves > (1ull << n))
        return fail(PIR_E_INVAL, "n_leaves=%llu outside [1, 2^%u]", (unsigned long long)n_leaves, n);
    if (sel_stride % 4 != 0 || sel_stride < 4 * words_for(n_leaves))
        return fail(PIR_E_INVAL, "sel_stride %llu must be a multiple of 4 and >= %llu",
                    (unsigned long long)sel_stride, (unsigned long long)(4 * words_for(n_leaves)));
    if ((uintptr_t)d_keys % 16 != 0) return fail(PIR_E_INVAL, "d_keys must be 16-byte aligned");
    if ((uintptr_t)d_sel % 4 != 0) return fail(PIR_E_INVAL, "d_sel must be 4-byte aligned");
    int rc = ctx->bind();
    if (rc) return rc;
    return eval_groups(ctx, (const uint8_t*)d_keys, n, n_keys, n_leaves, (uint32_t*)d_sel, sel_stride / 4,
                       (hipStream_t)hip_stream);
}

int pir_dpf_dpxor_async(pir_db* d, const void* d_keys, uint32_t n_keys, void* d_out, void* hip_stream) {
    clear_error();
    Db* db = reinterpret_cast<Db*>(d);
    if (!db || !d_keys || !d_out) return fail(PIR_E_INVAL, "pir_dpf_dpxor_async: NULL argument");
    if (n_keys == 0 || n_keys > PIR_MAX_BATCH)
        return fail(PIR_E_INVAL, "n_keys=%u outside [1, %u]", n_keys, PIR_MAX_BATCH);
    if ((uintptr_t)d_keys % 16 != 0) return fail(PIR_E_INVAL, "d_keys must be 16-byte aligned");
    const Geometry& g = db->geo;
    const uint32_t n = pir_dpf_domain_bits(g.n);
    if (n > kMaxDomainBits) return fail(PIR_E_INVAL, "database domain 2^%u too large", n);
    Ctx* ctx = db->ctx;
    int rc = ctx->bind();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    // selection rows: the scan's row pitch, whole 256-byte lines
    const uint64_t stride = (4 * g.nb + 255) / 256 * 256;
    uint64_t gq = kSelScratchBudget / stride;
    if (gq < 1) gq = 1;
    if (gq > n_keys) gq = n_keys;
    DevBuf *sb, *pb;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        sb = &ctx->dpf_ws[s].sel;
        pb = &ctx->workspaces[s];
    }
    if ((rc = grow(*sb, (size_t)gq * stride, s, "DPF selection workspace"))) return rc;
    const uint64_t kb = dpf_key_bytes(n);
    for (uint32_t q0 = 0; q0 < n_keys; q0 += (uint32_t)gq) {
        const uint32_t q = n_keys - q0 < gq ? n_keys - q0 : (uint32_t)gq;
        Plan p;
        if ((rc = ctx->plan_for(*db, q, nullptr, p))) return rc;
        const size_t need = partial_bytes(g, p, q);
        if ((rc = grow(*pb, need + need / 4, s, "workspace allocation"))) return rc;
        if ((rc = eval_groups(ctx, (const uint8_t*)d_keys + (uint64_t)q0 * kb, n, q, g.n, (uint32_t*)sb->ptr,
                              stride / 4, s)))
            return rc;
        if ((rc = ctx->launch_scan(*db, p, (const uint32_t*)sb->ptr, stride / 4, q,
                                    (uint8_t*)d_out + (uint64_t)q0 * g.R, (uint8_t*)pb->ptr, s)))
            return rc;
    }
    return PIR_OK;
}

}  // extern "C"
