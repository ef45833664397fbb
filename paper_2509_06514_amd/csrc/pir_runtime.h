// Runtime objects behind the opaque C handles.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "pir_internal.h"

namespace pir {

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
void clear_error();

// Growable device buffer (contents are not preserved on growth).
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void reset();
    hipError_t ensure(size_t want);
};

// Host rows (src, src_stride bytes apart, row_bytes each) laid out at a
// pitch of dstride bytes, each row's tail zero: pack_range writes bytes
// [off, off + len) of that layout to dst[0, len), pack_rows its first nr
// rows.  Copies of 8 MiB or more are split over up to 8 host threads; a
// thread that cannot be started leaves its share to the caller's thread.
void pack_range(uint8_t* dst, const uint8_t* src, uint64_t src_stride, uint64_t row_bytes, uint64_t dstride,
                uint64_t off, uint64_t len);
void pack_rows(uint8_t* dst, const uint8_t* src, uint32_t nr, uint64_t src_stride, uint64_t row_bytes,
               uint64_t dstride);

// Growable pinned host buffer.
struct HostBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf();
    void reset();
    hipError_t ensure(size_t want);
};

// Execution slot for the synchronous calls: a stream with its own staging
// and scratch buffers.
struct Exec {
    hipStream_t stream = nullptr;
    bool busy = false;
    HostBuf h_sel, h_out;
    DevBuf d_sel, d_out, partials;
    hipEvent_t staged[2] = {nullptr, nullptr};  // uploads out of the two staging halves
};

// Host rows -> device layout and device answers -> host, for the synchronous
// calls, all on ex->stream.  upload_rows copies q rows of row_bytes bytes
// (src_stride apart) to dst at a pitch of dstride: pinned rows with one
// pitched copy (the device rows' tails past row_bytes are then left as they
// were), pageable rows packed, tails zeroed, into two pinned staging halves
// of at most 16 MiB in turn, so that packing one piece overlaps the upload
// of the one before.  download_answers copies bytes from src to out and
// waits for the stream: straight into a pinned out, else through ex->h_out.
int upload_rows(Exec* ex, const uint8_t* src, uint64_t src_stride, uint64_t row_bytes, uint32_t q, uint8_t* dst,
                uint64_t dstride, const char* what);
int download_answers(Exec* ex, const void* src, uint8_t* out, size_t bytes, const char* what);

struct TimedPair {
    hipEvent_t a, b;
    int stage;
};

struct Ctx;

struct Db {
    Ctx* ctx = nullptr;
    Geometry geo;
    DevBuf data;                    // bit-sliced records
    hipStream_t ctx_stream = nullptr;  // load / update / tuning
    std::mutex mu;                  // serialises updates and reads
};

// Per-stream scratch of the DPF calls: tree levels, and the selection rows
// the key-to-answer path hands from the evaluation to the scan.
struct DpfWs {
    DevBuf nodes, sel;
};

// A captured scan (stage 1 + stage 2) for one database buffer, plan, query
// count and set of device pointers, instantiated once and replayed.
struct GraphKey {
    const void* data;
    uint64_t n;
    uint32_t R, variant, qt, unroll, groups, q;
    const void* sel;
    uint64_t stride_words;
    const void* out;
    const void* partials;
    bool operator<(const GraphKey& o) const;
};
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* db = nullptr;
    uint64_t last_use = 0;
};

// Tune-cache key: (record bytes, query-count bucket = Q rounded up to a power
// of two, log2 of the block count rounded down); the architecture is fixed
// (gfx950).  A plain struct, so that a lookup allocates nothing.
struct TuneKey {
    uint32_t R, qb, nbits;
    bool operator<(const TuneKey& o) const;
    std::string str(const std::string& arch) const;  // "gfx950/R32/Q64/NB23" (cache file form)
};

struct Ctx {
    int device = 0;
    std::string arch;
    int n_cu = 0;
    std::mutex mu;
    std::vector<std::unique_ptr<Exec>> pool;
    std::unordered_map<hipStream_t, DevBuf> workspaces;  // per caller stream
    std::unordered_map<hipStream_t, DpfWs> dpf_ws;       // per caller stream
    std::map<TuneKey, pir_kernel_cfg> tuned;
    void* noalloc_scratch = nullptr;  // this device's fixed scan scratch (pir_noalloc.hip)
    std::atomic<bool> timing_on{false};
    std::atomic<bool> graphs_on{true};
    std::mutex graph_mu;                  // guards `graphs`
    std::mutex capture_mu;                // one capture at a time on capture_stream
    hipStream_t capture_stream = nullptr;
    std::map<GraphKey, GraphEntry> graphs;
    uint64_t graph_clock = 0;
    std::vector<TimedPair> pending;
    std::vector<hipEvent_t> free_events;
    pir_timing acc{};

    ~Ctx();
    int bind();
    int acquire(Exec** out);
    void release(Exec* e);
    hipEvent_t take_event();
    int plan_for(const Db& db, uint32_t q, const pir_kernel_cfg* cfg, Plan& p);
    // records (a, b) as a timed interval of `stage` (1, 2: scan stages; 3: DPF evaluation;
    // 4: F_p main kernel)
    void add_timed(hipEvent_t a, hipEvent_t b, int stage);
    int enqueue_scan(const Db& db, const Plan& p, const uint32_t* d_sel, uint64_t stride_words, uint32_t q,
                     uint8_t* d_out, uint8_t* partials, hipStream_t s);
    // enqueue_scan through the graph cache (eager while timing is on or graphs are off)
    int launch_scan(const Db& db, const Plan& p, const uint32_t* d_sel, uint64_t stride_words, uint32_t q,
                    uint8_t* d_out, uint8_t* partials, hipStream_t s);
    void drop_graphs(const void* db);  // all graphs of a database (nullptr: every graph)
    TuneKey tune_key(const Geometry& g, uint32_t q) const;
    void save_tune_cache();
    void load_tune_cache();
};

int finish_plan(const Geometry& g, uint32_t q, Plan& p);
int check_async_args(Db* db, const void* d_sel, uint64_t sel_stride, uint32_t q, void* d_out);

// The fixed scan scratch of the no-allocation entry point (pir_noalloc.hip):
// its device address on the current device, looked up once per device.
int noalloc_scratch_for_current_device(void** out);

// DPF evaluation of n_keys device keys into selection rows on stream s, with
// the stream's node scratch (pir_dpf_api.cpp); and the most scratch that
// call may allocate.
int dpf_eval_into(Ctx* ctx, const uint8_t* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves, uint32_t* d_sel,
                  uint64_t stride_words, hipStream_t s);
uint64_t dpf_eval_scratch_bytes(uint32_t n, uint64_t n_leaves, uint32_t n_keys);
size_t partial_bytes(const Geometry& g, const Plan& p, uint32_t q);

}  // namespace pir
