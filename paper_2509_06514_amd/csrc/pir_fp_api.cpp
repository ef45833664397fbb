// C ABI of the F_p inner-product form (IM-PIR Sec. 2: a database over
// F_p^{N x L}; the answer is the inner product of the query vector with it).
// The database lives in its own handle type so it can never reach the XOR
// scan by mistake.
#include <algorithm>
#include <cstring>
#include <memory>

#include "pir_runtime.h"

namespace pir {

struct FpDb {
    Ctx* ctx = nullptr;
    uint64_t n = 0;      // records
    uint32_t L = 0;      // elements per record
    uint32_t lpad = 0;   // L rounded up to 16
    uint32_t p = 0, magic = 0;
    uint64_t tiles = 0;  // ceil(n / 64)
    DevBuf data;
    hipStream_t stream = nullptr;
    std::mutex mu;
    uint64_t bytes() const { return tiles * 64ull * lpad; }
};

namespace {

constexpr uint64_t kChunkBytes = 256ull << 20;  // load / read staging

uint64_t chunk_records(uint32_t L) {
    uint64_t r = kChunkBytes / L / 64 * 64;
    return r < 64 ? 64 : r;
}

// Workgroups a launch aims for (record groups x query tiles x column groups).
constexpr uint64_t kFpTargetWorkgroups = 2048;

// Plan for q queries: row tiles of 16 queries (up to 4), column tiles of 16
// elements (up to 4), record groups so that about kFpTargetWorkgroups
// workgroups run, each group an even number of tiles.
void fp_plan(const FpDb& db, uint32_t q, FpParams& a, uint32_t& rt, uint32_t& ct) {
    rt = q <= 16 ? 1 : q <= 32 ? 2 : 4;
    const uint32_t n_ct = db.lpad / 16;
    ct = n_ct >= 4 ? 4 : n_ct >= 2 ? 2 : 1;
    a.tiles = db.tiles;
    a.L = db.L;
    a.lpad = db.lpad;
    a.n_ct = n_ct;
    a.n_qt = (q + 16 * rt - 1) / (16 * rt);
    a.n_cg = (n_ct + ct - 1) / ct;
    a.q_total = q;
    a.p = db.p;
    a.magic = db.magic;
    uint64_t g = (kFpTargetWorkgroups + a.n_qt * a.n_cg - 1) / (a.n_qt * a.n_cg);
    g = std::max<uint64_t>(g, (db.tiles + kFpMaxTilesPerGroup - 1) / kFpMaxTilesPerGroup);
    g = std::min<uint64_t>(g, db.tiles);
    a.tiles_per_group = (db.tiles + g - 1) / g;
    // even, so that every wave step starts on a 128-byte line of the query rows
    a.tiles_per_group = std::min<uint64_t>((a.tiles_per_group + 1) & ~1ull, kFpMaxTilesPerGroup);
    a.groups = (uint32_t)((db.tiles + a.tiles_per_group - 1) / a.tiles_per_group);
}

int enqueue_fp(FpDb& db, const uint8_t* d_v, uint64_t v_stride, uint32_t q, uint8_t* d_out, DevBuf& ws,
               hipStream_t s, bool may_sync) {
    FpParams a;
    uint32_t rt, ct;
    fp_plan(db, q, a, rt, ct);
    a.v_stride = v_stride;
    const size_t part_bytes = ((size_t)a.groups * q * db.L + 255) / 256 * 256;
    const size_t need = part_bytes + fp_stage2_tmp_bytes(a.groups, (uint64_t)q * db.L);
    if (need > ws.bytes) {
        if (ws.ptr && may_sync) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail(e, "workspace sync");
        }
        hipError_t e = ws.ensure(need + need / 4);
        if (e != hipSuccess) return hip_fail(e, "workspace allocation");
    }
    Ctx* ctx = db.ctx;
    const bool timed = ctx->timing_on.load();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        e0 = ctx->take_event();
        e1 = ctx->take_event();
    }
    if (e0) (void)hipEventRecord(e0, s);
    hipError_t e = launch_fp_stage1((const uint8_t*)db.data.ptr, d_v, (uint8_t*)ws.ptr, a, rt, ct, s);
    if (e != hipSuccess) return hip_fail(e, "F_p stage-1 launch");
    if (e1) (void)hipEventRecord(e1, s);
    e = launch_fp_stage2((const uint8_t*)ws.ptr, a.groups, (uint64_t)q * db.L, db.p, db.magic,
                         (uint32_t*)((uint8_t*)ws.ptr + part_bytes), d_out, s);
    if (e != hipSuccess) return hip_fail(e, "F_p stage-2 launch");
    if (timed && e0 && e1) ctx->add_timed(e0, e1, 4);
    return PIR_OK;
}

}  // namespace
}  // namespace pir

using namespace pir;

extern "C" {

int pir_fp_db_load(pir_ctx* c, const void* elements, uint64_t n_records, uint32_t record_elems, uint32_t p,
                   pir_fpdb** out) {
    clear_error();
    if (!c || !elements || !out) return fail(PIR_E_INVAL, "pir_fp_db_load: NULL argument");
    *out = nullptr;
    if (n_records == 0 || record_elems == 0) return fail(PIR_E_INVAL, "pir_fp_db_load: N and L must be positive");
    if (record_elems > 65536) return fail(PIR_E_INVAL, "pir_fp_db_load: L > 65536");
    if (p < 2 || p > 127) return fail(PIR_E_INVAL, "pir_fp_db_load: p=%u outside [2, 127]", p);
    if (n_records > (1ull << 36)) return fail(PIR_E_INVAL, "pir_fp_db_load: N too large");
    const uint8_t* src = (const uint8_t*)elements;
    {
        // every element must be a field element (a value below p)
        uint8_t bad = 0;
        const uint64_t total = n_records * record_elems;
        for (uint64_t i = 0; i < total; ++i) bad |= (uint8_t)(src[i] >= p);
        if (bad) return fail(PIR_E_INVAL, "pir_fp_db_load: an element is >= p");
    }
    Ctx* ctx = reinterpret_cast<Ctx*>(c);
    int rc = ctx->bind();
    if (rc) return rc;
    auto db = std::make_unique<FpDb>();
    db->ctx = ctx;
    db->n = n_records;
    db->L = record_elems;
    db->lpad = (record_elems + 15) / 16 * 16;
    db->p = p;
    db->magic = (uint32_t)((1ull << 32) / p);
    db->tiles = (n_records + 63) / 64;
    hipError_t e = hipStreamCreateWithFlags(&db->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    auto cleanup = [&](int code) {
        db->data.reset();
        (void)hipStreamDestroy(db->stream);
        return code;
    };
    if ((e = db->data.ensure(db->bytes())) != hipSuccess)
        return cleanup(fail(PIR_E_NOMEM, "pir_fp_db_load: cannot allocate %llu bytes of HBM",
                            (unsigned long long)db->bytes()));
    DevBuf stage;
    const uint64_t per = std::min<uint64_t>(chunk_records(record_elems), n_records);
    if ((e = stage.ensure(per * record_elems)) != hipSuccess) return cleanup(hip_fail(e, "staging allocation"));
    for (uint64_t r0 = 0; r0 < n_records; r0 += per) {
        const uint64_t nr = std::min(per, n_records - r0);
        e = hipMemcpyAsync(stage.ptr, src + r0 * record_elems, nr * record_elems, hipMemcpyHostToDevice, db->stream);
        if (e == hipSuccess)
            e = launch_fp_tile((const uint8_t*)stage.ptr, nr, record_elems, db->lpad,
                               (uint8_t*)db->data.ptr + (r0 / 64) * 64ull * db->lpad, db->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(db->stream);
        if (e != hipSuccess) return cleanup(hip_fail(e, "F_p database upload"));
    }
    *out = reinterpret_cast<pir_fpdb*>(db.release());
    return PIR_OK;
}

int pir_fp_db_free(pir_fpdb* d) {
    clear_error();
    if (!d) return fail(PIR_E_INVAL, "pir_fp_db_free: NULL");
    FpDb* db = reinterpret_cast<FpDb*>(d);
    (void)db->ctx->bind();
    (void)hipStreamSynchronize(db->stream);
    db->data.reset();
    (void)hipStreamDestroy(db->stream);
    delete db;
    return PIR_OK;
}

uint64_t pir_fp_min_v_stride(const pir_fpdb* d) {
    if (!d) return 0;
    return reinterpret_cast<const FpDb*>(d)->tiles * 64;
}

// Query-row pitch for the scan: the smallest odd multiple of 128 bytes that
// holds a row.  A wave's loads touch 64 rows at once; at a power-of-two pitch
// of many MiB those rows share every low address bit and so crowd the same
// HBM channels and banks, which an odd multiple of 128 avoids.
static uint64_t fp_pitch(uint64_t min_bytes) {
    const uint64_t lines = (min_bytes + 127) / 128;
    return 128 * (lines | 1);
}

uint64_t pir_fp_v_stride(const pir_fpdb* d) {
    if (!d) return 0;
    return fp_pitch(reinterpret_cast<const FpDb*>(d)->tiles * 64);
}

int pir_fp_db_read(pir_fpdb* d, uint64_t first, uint64_t count, void* out_elements) {
    clear_error();
    if (!d || !out_elements) return fail(PIR_E_INVAL, "pir_fp_db_read: NULL argument");
    FpDb* db = reinterpret_cast<FpDb*>(d);
    if (count == 0) return PIR_OK;
    if (first >= db->n || count > db->n - first) return fail(PIR_E_INVAL, "pir_fp_db_read: range outside N");
    int rc = db->ctx->bind();
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(db->mu);
    const uint64_t per = chunk_records(db->L);
    DevBuf stage;
    hipError_t e = stage.ensure(std::min<uint64_t>(per, (count + 127) / 64 * 64) * db->L);
    if (e != hipSuccess) return hip_fail(e, "staging allocation");
    uint64_t r = first;
    while (r < first + count) {
        const uint64_t r0 = r / 64 * 64;  // chunk starts on a tile
        const uint64_t r1 = std::min({r0 + per, db->n, first + count});
        e = launch_fp_untile((const uint8_t*)db->data.ptr + (r0 / 64) * 64ull * db->lpad, r1 - r0, db->L, db->lpad,
                             (uint8_t*)stage.ptr, db->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((uint8_t*)out_elements + (r - first) * db->L, (uint8_t*)stage.ptr + (r - r0) * db->L,
                               (r1 - r) * db->L, hipMemcpyDeviceToHost, db->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(db->stream);
        if (e != hipSuccess) return hip_fail(e, "F_p read-back");
        r = r1;
    }
    return PIR_OK;
}

int pir_fp_inner_async(pir_fpdb* d, const void* d_v, uint64_t v_stride, uint32_t q, void* d_out, void* hip_stream) {
    clear_error();
    FpDb* db = reinterpret_cast<FpDb*>(d);
    if (!db || !d_v || !d_out) return fail(PIR_E_INVAL, "pir_fp_inner_async: NULL argument");
    if (q == 0 || q > PIR_MAX_BATCH) return fail(PIR_E_INVAL, "q=%u outside [1, %u]", q, PIR_MAX_BATCH);
    if (v_stride % 16 != 0 || v_stride < db->tiles * 64)
        return fail(PIR_E_INVAL, "v_stride %llu must be a multiple of 16 and >= %llu", (unsigned long long)v_stride,
                    (unsigned long long)(db->tiles * 64));
    if ((uintptr_t)d_v % 16 != 0) return fail(PIR_E_INVAL, "d_v must be 16-byte aligned");
    Ctx* ctx = db->ctx;
    int rc = ctx->bind();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    DevBuf* ws;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ws = &ctx->workspaces[s];
    }
    return enqueue_fp(*db, (const uint8_t*)d_v, v_stride, q, (uint8_t*)d_out, *ws, s, true);
}

int pir_fp_inner(pir_fpdb* d, const uint8_t* v, uint64_t v_stride, uint32_t q, uint8_t* out) {
    clear_error();
    FpDb* db = reinterpret_cast<FpDb*>(d);
    if (!db || !v || !out) return fail(PIR_E_INVAL, "pir_fp_inner: NULL argument");
    if (q == 0 || q > PIR_MAX_BATCH) return fail(PIR_E_INVAL, "q=%u outside [1, %u]", q, PIR_MAX_BATCH);
    if (v_stride < db->n) return fail(PIR_E_INVAL, "v_stride %llu < N", (unsigned long long)v_stride);
    Ctx* ctx = db->ctx;
    int rc = ctx->bind();
    if (rc) return rc;
    Exec* ex = nullptr;
    if ((rc = ctx->acquire(&ex))) return rc;
    struct Releaser {
        Ctx* c;
        Exec* e;
        ~Releaser() { c->release(e); }
    } rel{ctx, ex};
    const uint64_t dstride = fp_pitch(db->tiles * 64);
    const size_t v_bytes = (size_t)dstride * q, out_bytes = (size_t)q * db->L;
    hipError_t e;
    if ((e = ex->d_sel.ensure(v_bytes)) != hipSuccess) return hip_fail(e, "device query buffer");
    if ((e = ex->d_out.ensure(out_bytes)) != hipSuccess) return hip_fail(e, "device answer buffer");
    // a pinned caller's rows are copied as they are, so the device rows' tails
    // past N keep older bytes: they meet the zero padding records of the last
    // tile only and add nothing
    if ((rc = upload_rows(ex, v, v_stride, db->n, q, (uint8_t*)ex->d_sel.ptr, dstride, "query upload"))) return rc;
    if ((rc = enqueue_fp(*db, (const uint8_t*)ex->d_sel.ptr, dstride, q, (uint8_t*)ex->d_out.ptr, ex->partials,
                         ex->stream, true)))
        return rc;
    return download_answers(ex, ex->d_out.ptr, out, out_bytes, "F_p inner product");
}

}  // extern "C"
