/*
 * pir.h -- C ABI of the MI355X dpXOR library (libpir.so).
 *
 * dpXOR is the server-side hot path of DPF-based two-server private
 * information retrieval (IM-PIR, Sec. 2 "Multi-Server PIR" and Sec. 3.3
 * "PIR linear operations"): given a resident database D of N records of R
 * bytes and a selection bit vector v in F_2^N (a DPF key share expanded over
 * the whole domain, v[j] = Eval(k, j)), the server returns
 *
 *     r = XOR over j = 0 .. N-1 of v[j] * D[j]          (an R-byte record)
 *
 * The client XORs the two servers' answers to recover D[i].
 *
 * Conventions shared by every call:
 *  - Record j is bytes [j*R, (j+1)*R) of a row-major host buffer.
 *  - Bit j of a selection vector is (sel[j >> 3] >> (j & 7)) & 1 (LSB first).
 *    Bits at positions >= N are ignored (they may hold anything).
 *  - A batch of Q selection vectors is Q rows `sel_stride` bytes apart; row q
 *    of the answer is r for row q alone (queries are independent, Sec. 3.4).
 *  - Every call returns PIR_OK (0) or a negative pir_status; on failure
 *    nothing is half done (a failed load frees what it allocated) and
 *    pir_last_error() returns a message for the calling thread.
 *  - There is no CPU fallback: without a usable gfx950 device, calls fail
 *    with PIR_E_DEVICE.
 */
#ifndef PIR_H
#define PIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pir_ctx pir_ctx;
typedef struct pir_db pir_db;
typedef struct pir_server pir_server;
typedef struct pir_fpdb pir_fpdb;

typedef enum pir_status {
    PIR_OK = 0,
    PIR_E_INVAL = -1,    /* bad argument: NULL, N = 0, R = 0, size overflow, Q out of range */
    PIR_E_NOMEM = -2,    /* device or pinned allocation failed, or over the HBM budget */
    PIR_E_DEVICE = -3,   /* a HIP call failed; the message names it */
    PIR_E_BUSY = -4,     /* a serving queue is full */
    PIR_E_NOTFOUND = -5, /* unknown database id or ticket */
    PIR_E_SHUTDOWN = -6, /* the server is shutting down; the request was not run */
    PIR_E_TIMEOUT = -7   /* pir_serve_wait timed out; the request is still pending */
} pir_status;

/* Largest batch a single call accepts. */
#define PIR_MAX_BATCH 4096u

/* Kernel variants for the batched scan (pir_kernel_cfg.variant). */
#define PIR_VARIANT_AUTO 0u     /* autotuned choice (cached per shape) */
#define PIR_VARIANT_VALU 1u     /* bitwise select-XOR on the vector ALUs */
#define PIR_VARIANT_MFMA_I8 2u  /* GF(2) contraction on int8 MFMA, exact int32, then mod 2 */
#define PIR_VARIANT_MFMA_F4 3u  /* GF(2) contraction on fp4 MFMA, exact fp32 counts, then mod 2 */

/* Thread-local description of the last failure on this thread ("" if none). */
const char* pir_last_error(void);

/* Library version string. */
const char* pir_version(void);

/* ---------------------------------------------------------------- context */

/* Bind to HIP device `hip_device` (must be gfx950).  The context owns the
 * streams, workspaces and pinned staging buffers used by the sync calls. */
int pir_ctx_create(int hip_device, pir_ctx** out);
int pir_ctx_destroy(pir_ctx* ctx);

/* ---------------------------------------------------------------- database */

/*
 * Database preload (IM-PIR Sec. 3.3 "Database preloading": the database is
 * resident before any query and its transfer is not part of a query).
 * Copies n_records x record_bytes bytes from the host buffer `records` into
 * HBM.  The caller may free `records` on return; the library owns the device
 * copy until pir_db_free.  The device copy is stored bit-sliced: each block
 * of 32 consecutive records becomes 8*R 32-bit words, word b holding bit b of
 * the 32 records, with records past N zero.  Record 32*blk+i sits at bit i,
 * except that inside every 4-bit group records 4n and 4n+2 trade places.
 * Errors: PIR_E_INVAL (NULL, N = 0, R = 0, N*R overflow), PIR_E_NOMEM.
 */
int pir_db_load(pir_ctx* ctx, const void* records, uint64_t n_records, uint32_t record_bytes,
                pir_db** out);

/*
 * Bulk update of records [first, first + count) from a host buffer (the
 * idle-window update of Sec. 3.3).  Must not overlap a scan of the same
 * database; it synchronises with the context's own calls only.
 */
int pir_db_update(pir_db* db, uint64_t first, uint64_t count, const void* records);

/* Copy records [first, first + count) back to the host in row-major form. */
int pir_db_read(pir_db* db, uint64_t first, uint64_t count, void* out_records);

int pir_db_free(pir_db* db);

typedef struct pir_db_info {
    uint64_t n_records;     /* N */
    uint32_t record_bytes;  /* R */
    uint32_t reserved;
    uint64_t n_blocks;      /* ceil(N / 32) bit-sliced blocks */
    uint64_t device_bytes;  /* HBM held by the database */
    uint64_t sel_words;     /* 32-bit selection words per query row (= n_blocks) */
} pir_db_info;

int pir_db_get_info(const pir_db* db, pir_db_info* out);

/* Minimum device selection-row stride in bytes for the async calls:
 * 4 * ceil(N / 32), i.e. whole 32-bit words covering every block. */
uint64_t pir_db_min_sel_stride(const pir_db* db);

/* ---------------------------------------------------------------- scans */

/*
 * One query, synchronous: sel_bits is a host buffer of ceil(N/8) bytes;
 * out_record receives R bytes.  Uploads the selection, runs the scan and
 * downloads the answer on a pooled stream; safe to call from several threads
 * on the same database.
 */
int pir_dpxor(pir_db* db, const uint8_t* sel_bits, uint8_t* out_record);

/*
 * Q queries in one database pass, synchronous.  sel_bits holds q rows
 * sel_stride bytes apart (sel_stride >= ceil(N/8)); out receives q rows of R
 * bytes.  1 <= q <= PIR_MAX_BATCH.  Pinned buffers (pir_host_alloc) are
 * copied to and from the device directly; pageable ones go through the
 * library's pinned staging, in chunks whose packing overlaps the upload.
 */
int pir_dpxor_batch(pir_db* db, const uint8_t* sel_bits, uint64_t sel_stride, uint32_t q,
                    uint8_t* out);

/*
 * Q queries, asynchronous on a caller stream, device buffers only (for
 * example torch tensors).  d_sel: q rows of 32-bit words, sel_stride bytes
 * apart, sel_stride a multiple of 4 and >= pir_db_min_sel_stride(db), base
 * 4-byte aligned; bits of blocks past N are ignored.  d_out: q*R bytes.
 * hip_stream: a hipStream_t (NULL = the null stream).  The call enqueues the
 * scan and the cross-workgroup reduction and returns; d_out is valid once the
 * stream reaches that point.  The library keeps one scratch workspace per
 * stream, so overlapping calls on one stream are ordered and safe; it may
 * synchronise the stream once to grow that workspace.
 */
int pir_dpxor_batch_async(pir_db* db, const void* d_sel, uint64_t sel_stride, uint32_t q,
                          void* d_out, void* hip_stream);

/*
 * The same scan for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, layout and results as pir_dpxor_batch_async; the partial
 * answers go to a fixed per-device scratch array of
 * PIR_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it
 * runs on until the process ends (its address is looked up when a context
 * is created on the device), instead of a library-allocated workspace.  The
 * call allocates nothing, records no events and captures no graph: it
 * enqueues the scan's two kernels on hip_stream.  When the plan's partials
 * (record groups x q x R rounded up to 4 bytes) exceed the scratch, the
 * records are taken in fewer, longer groups (same answers); if even the
 * fewest groups the exact matrix-core counts allow do not fit (about
 * q * R > 32 MiB), the call fails with PIR_E_INVAL and a message naming the
 * limit.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on the device (on other streams, or from other host threads without
 * ordering) race on it and must not be issued; calls on one stream are
 * ordered and safe.  Nothing in the array needs clearing between calls.
 */
#define PIR_NOALLOC_SCRATCH_BYTES (32u << 20)
int pir_dpxor_batch_async_noalloc(pir_db* db, const void* d_sel, uint64_t sel_stride, uint32_t q, void* d_out,
                                  void* hip_stream);

/* Explicit kernel configuration (tests of tile invariance, the autotuner). */
typedef struct pir_kernel_cfg {
    uint32_t variant; /* PIR_VARIANT_* */
    uint32_t q_tile;  /* queries per workgroup tile (variant-specific; 0 = default) */
    uint32_t unroll;  /* VALU: blocks per wave iteration; MFMA: 2/3/4 = LDS ring of that
                         many stages, 12 = split-K kernel on a 2-stage ring (fp4, q_tile 64),
                         15 = split-K kernel on a 2-stage ring whose selection words arrive
                         4 K-steps at a time, 16 = the same with wave-private database
                         stages, 17 = the same with the database words loaded straight
                         into registers (all fp4, q_tile 64; 17 runs as 16 where a record
                         group spans 4 GiB or more of the database, and 15-17 run as 12
                         where selection rows are not 16-byte aligned or lie more than
                         about 1.4 GB apart); 0 = default */
    uint32_t groups;  /* record groups = partial results per query (0 = default) */
} pir_kernel_cfg;

/* As pir_dpxor_batch_async, with an explicit configuration.  Unsupported
 * combinations return PIR_E_INVAL. */
int pir_dpxor_batch_async_cfg(pir_db* db, const void* d_sel, uint64_t sel_stride, uint32_t q,
                              void* d_out, void* hip_stream, const pir_kernel_cfg* cfg);

/* Configuration the library would use for q queries on db (after tuning). */
int pir_get_cfg(pir_db* db, uint32_t q, pir_kernel_cfg* out);

/*
 * Autotuner: times each candidate configuration for q queries on this
 * database (device-resident scratch selections of random-looking bits at a
 * 256-byte row pitch: the scan's time depends on the bits it multiplies,
 * not only on the bytes it reads), keeps the fastest in the
 * context's cache, keyed by (architecture, R, Q bucket, N bucket), and
 * writes the cache to the JSON file named by the PIR_TUNE_CACHE environment
 * variable if set.  Returns the chosen configuration in *out (may be NULL).
 */
int pir_tune(pir_db* db, uint32_t q, pir_kernel_cfg* out);

/*
 * Graph replay (on by default): the scan's launches (stage 1 + stage 2) are
 * captured once per (database buffer, plan, query count, device pointers)
 * into a hipGraph on a private stream and replayed with one graph launch on
 * the caller's stream; pir_dpxor, pir_dpxor_batch, the asynchronous calls,
 * the key-to-answer path and the server all go through this cache (up to 256
 * graphs per context, least recently used evicted; a database's graphs are
 * dropped when it is freed).  While timing is enabled the launches are
 * enqueued one by one instead, so that each stage can be timed.  on = 0
 * turns replay off for this context.
 */
int pir_graphs_enable(pir_ctx* ctx, int on);

/* ---------------------------------------------------------------- timing */

/*
 * Kernel timing: while enabled, the library records HIP events on the
 * launch stream around every scan kernel (stage 1) and reduction kernel
 * (stage 2) it launches.  pir_timing_read waits for the recorded events and
 * returns the launch counts and summed durations since the last reset.
 */
typedef struct pir_timing {
    uint64_t stage1_launches;
    double stage1_ms;
    uint64_t stage2_launches;
    double stage2_ms;
    uint64_t dpf_evals;       /* DPF evaluations (each a chain of expansion kernels) */
    double dpf_ms;            /* their summed durations, first launch to last */
    uint64_t fp_launches;     /* F_p inner-product main kernels */
    double fp_ms;
} pir_timing;

int pir_timing_enable(pir_ctx* ctx, int on);
int pir_timing_read(pir_ctx* ctx, pir_timing* out, int reset);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous-batching server (IM-PIR Sec. 3.4 "Batching client queries":
 * queries queue up and are dispatched to execution resources as they free
 * up).  Several databases stay resident; requests are queued per database;
 * a scheduler thread packs up to q_max pending requests of one database into
 * a free slot (its own stream, pinned buffers and workspace) and launches
 * one batched scan; requests that arrive meanwhile join later batches.
 * Slots run concurrently on the device.
 */
typedef struct pir_serve_config {
    uint64_t hbm_budget_bytes; /* admission limit for resident databases + slot buffers (0 = no limit) */
    uint32_t q_max;            /* largest batch per launch (<= PIR_MAX_BATCH; 0 = 64) */
    uint32_t max_wait_us;      /* a partial batch waits at most this long for company (0 = dispatch at once) */
    uint32_t n_slots;          /* concurrent in-flight batches (0 = 4) */
    uint32_t queue_cap;        /* queued (not yet dispatched) requests per database and kind before
                                  PIR_E_BUSY (0 = 65536) */
    uint32_t submit_wait_ms;   /* longest a submit waits for a free row of the pinned request ring
                                  before PIR_E_BUSY (0 = 1000) */
    uint64_t ring_bytes;       /* pinned selection ring per database (0 = 256 MiB); it holds at least
                                  (n_slots + 1) * q_max rows and at most queue_cap + n_slots * q_max */
} pir_serve_config;

typedef struct pir_serve_stats {
    uint64_t submitted;
    uint64_t completed;
    uint64_t rejected;        /* PIR_E_BUSY / PIR_E_SHUTDOWN at submit */
    uint64_t batches;
    double p50_us;            /* submit -> answer in host memory */
    double p99_us;
    double mean_us;
    double max_us;
    double elapsed_s;         /* since create or the last reset */
    double qps;               /* completed / elapsed_s */
    uint64_t batch_hist[13];  /* batches with size in [2^i, 2^(i+1)) */
    uint64_t h2d_bytes;       /* selection bytes uploaded */
    uint32_t max_inflight;    /* most slots busy at once (batches overlapping on the device) */
    uint32_t n_slots;
    uint64_t key_requests;    /* requests submitted as DPF keys */
    uint64_t updates_applied; /* record updates applied */
    uint64_t blocked_submits; /* submits that waited for a free ring row */
} pir_serve_stats;

int pir_serve_create(pir_ctx* ctx, const pir_serve_config* cfg, pir_server** out);

/* Admit a loaded database (PIR_E_NOMEM if it would exceed the budget).  The
 * database must outlive the server. */
int pir_serve_add_db(pir_server* srv, pir_db* db, uint32_t* db_id);

/*
 * Queue one query.  sel_bits (ceil(N/8) bytes) is copied into the
 * database's pinned request ring before the call returns; out (R bytes) must
 * stay valid until pir_serve_wait or pir_serve_poll reports completion.
 * Backpressure: when every ring row belongs to a queued or in-flight request
 * the call blocks until a batch retires (at most submit_wait_ms).  Errors:
 * PIR_E_NOTFOUND (db_id), PIR_E_BUSY (queue_cap requests already queued, or
 * no ring row freed within submit_wait_ms), PIR_E_SHUTDOWN.
 */
int pir_serve_submit(pir_server* srv, uint32_t db_id, const uint8_t* sel_bits, uint8_t* out,
                     uint64_t* ticket);

/*
 * Queue one query as a DPF key (IM-PIR Sec. 3.2): the server evaluates it
 * over the database's domain (n = pir_dpf_domain_bits(N)) and answers with
 * XOR_j Eval(key, j) * D[j].  key (pir_dpf_key_bytes(n) bytes, layout as in
 * the DPF section below) is copied before the call returns; out (R bytes)
 * must stay valid until completion.  Key requests are batched separately
 * from selection requests.  Errors as pir_serve_submit.
 */
int pir_serve_submit_key(pir_server* srv, uint32_t db_id, const uint8_t* key, uint8_t* out,
                         uint64_t* ticket);

/*
 * Replace records [first, first + count) of a served database (the paper
 * applies database updates in idle windows, on a stable version: Sec. 3.3).
 * The records (count * R bytes, row-major) are copied before the call
 * returns.  The update is ordered with the database's requests: every
 * request submitted before it is answered from the old records, every
 * request submitted after it from the new ones; it is applied once the
 * earlier requests have completed, and later requests wait for it.  The
 * ticket completes (pir_serve_wait / pir_serve_poll) when the records are in
 * place.  Errors: PIR_E_INVAL (range), PIR_E_NOTFOUND, PIR_E_SHUTDOWN.
 */
int pir_serve_update(pir_server* srv, uint32_t db_id, uint64_t first, uint64_t count, const void* records,
                     uint64_t* ticket);

/* Wait for a ticket: PIR_OK once out holds the answer, the request's own
 * error, PIR_E_TIMEOUT, or PIR_E_NOTFOUND for an unknown or already
 * collected ticket.  timeout_ms < 0 waits forever. */
int pir_serve_wait(pir_server* srv, uint64_t ticket, int timeout_ms);

/* Non-blocking: 1 if done (result in *status), 0 if pending. */
int pir_serve_poll(pir_server* srv, uint64_t ticket, int* status);

int pir_serve_stats_get(pir_server* srv, pir_serve_stats* out, int reset);

/* Stop accepting requests, finish everything queued or in flight, join the
 * scheduler and free the slots.  Every ticket completes or reports
 * PIR_E_SHUTDOWN; none is lost. */
int pir_serve_destroy(pir_server* srv);

/* ---------------------------------------------------------------- DPF */

/*
 * Distributed point functions (IM-PIR Sec. 3.1 key generation, Sec. 3.2
 * evaluation, eq. 1-3) over a domain of 2^n leaves:
 *
 *   Eval(k, j) = R(n, j),   R(0, 0) = C0[0, 0],
 *   R(d, j) = PRF_{R(d-1, j/2)}(j mod 2) XOR C_{R(d-1, j/2) mod 2}[j mod 2, d].
 *
 * Node values are 16-byte blocks; "mod 2" is bit 0 of byte 0; PRF_s(x) is
 * AES-128 (FIPS-197) under key s of the block whose byte 0 is x and whose
 * other bytes are 0.  The selection bit of leaf j is bit 0 of byte 0 of
 * Eval(k, j); the two parties' bits differ exactly at alpha.
 *
 * Key layout (pir_dpf_key_bytes(n) = 64 * (n + 1) bytes): codeword C0 then
 * codeword C1, each 2 x (n+1) blocks; block [x][d] of codeword c at byte
 * ((2c + x) * (n + 1) + d) * 16.
 */
uint64_t pir_dpf_key_bytes(uint32_t n);

/* Smallest n with 2^n >= n_records (0 for n_records <= 1): the domain a
 * database's keys are generated for. */
uint32_t pir_dpf_domain_bits(uint64_t n_records);

/*
 * Client side, host only (no device is touched).  Writes the two parties'
 * keys for the point function that is 1 at alpha (alpha < 2^n, n <= 62):
 * the tree construction of Boyle, Gilboa and Ishai (CCS 2016) that the paper
 * refers to, in the codeword form above -- C0[0][0] is the party's root, all
 * other C0 blocks are zero, C1 holds the per-level correction words (equal in
 * both keys).  root0/root1: 16 bytes each that the caller draws from a
 * cryptographic random source; their bit 0 is replaced by the party index.
 * key0/key1: pir_dpf_key_bytes(n) bytes each, caller-owned.
 */
int pir_dpf_gen(uint64_t alpha, uint32_t n, const uint8_t* root0, const uint8_t* root1, uint8_t* key0,
                uint8_t* key1);

/*
 * Full-domain evaluation on the device, asynchronous on hip_stream.
 * d_keys: n_keys keys of pir_dpf_key_bytes(n) bytes, consecutive, 16-byte
 * aligned, device memory.  Row q of d_sel (rows sel_stride bytes apart,
 * sel_stride a multiple of 4 and >= 4 * ceil(n_leaves / 32), base 4-byte
 * aligned) receives words [0, ceil(n_leaves / 32)): bit j = Eval(k_q, j),
 * LSB first, for every j < min(2^n, 32 * ceil(n_leaves / 32)); the words
 * past that are not written.  1 <= n_leaves <= 2^n, n <= 36,
 * 1 <= n_keys <= PIR_MAX_BATCH.  The library keeps a scratch buffer per
 * stream for the tree levels (2 * ceil(n_leaves / 32) blocks per key in flight,
 * keys processed in groups of at most 1.5 GiB of scratch) and may synchronise
 * the stream once to grow it.  Errors: PIR_E_INVAL, PIR_E_NOMEM, PIR_E_DEVICE.
 */
int pir_dpf_eval_async(pir_ctx* ctx, const void* d_keys, uint32_t n, uint32_t n_keys, uint64_t n_leaves,
                       void* d_sel, uint64_t sel_stride, void* hip_stream);

/*
 * A server's whole answer from keys (Sec. 3.2 then Sec. 3.3): evaluates
 * n_keys keys for the database's domain (n = pir_dpf_domain_bits(N)) into a
 * library-owned selection workspace and scans the database with them in
 * batches; row q of d_out (n_keys * R bytes, device) = XOR over j < N of
 * Eval(k_q, j) * D[j].  Same key layout and alignment as pir_dpf_eval_async;
 * asynchronous on hip_stream, with the same workspace rules.  Databases of
 * more than 2^36 records (a domain past the evaluation's n <= 36) give
 * PIR_E_INVAL.
 */
int pir_dpf_dpxor_async(pir_db* db, const void* d_keys, uint32_t n_keys, void* d_out, void* hip_stream);

/*
 * Client side, host only: the record from the two servers' answers
 * (Algorithm 1, client step: D[i] = r1 XOR r2).  out may alias either
 * input.  Errors: PIR_E_INVAL for NULL pointers.
 */
int pir_reconstruct(const uint8_t* ans0, const uint8_t* ans1, uint64_t record_bytes, uint8_t* out);

/* ---------------------------------------------------------------- F_p */

/*
 * The answer over a prime field (IM-PIR Sec. 2 states the database as D in
 * F_p^{N x L} and the server's answer as the inner product of the query
 * vector with it; the XOR scan above is the case p = 2 on bits):
 *
 *     r_q[l] = ( sum over j < N of v_q[j] * D[j][l] ) mod p,   l < L.
 *
 * Elements are bytes: a record is L elements (one byte each, < p), a query
 * is N bytes, one per record.  2 <= p <= 127.  Query bytes must be below 128
 * (they are the integers they hold; values in [p, 128) are allowed and act
 * as their residues).  Answers are L bytes per query, each in [0, p).  Two
 * servers holding v and e_i - v (mod p) return answers that add to D[i]
 * (mod p).
 */

/* Copy N records of L elements (row-major, N*L bytes) into HBM.  Fails with
 * PIR_E_INVAL if an element is >= p, N or L is 0, or p is outside [2, 127].
 * The database must be freed before its context. */
int pir_fp_db_load(pir_ctx* ctx, const void* elements, uint64_t n_records, uint32_t record_elems, uint32_t p,
                   pir_fpdb** out);
int pir_fp_db_free(pir_fpdb* db);

/* Records [first, first + count) back in row-major order. */
int pir_fp_db_read(pir_fpdb* db, uint64_t first, uint64_t count, void* out_elements);

/* Smallest query row pitch for the device call: N rounded up to 64 (0 for
 * NULL).  Bytes of a row past N are read and meet zero records. */
uint64_t pir_fp_min_v_stride(const pir_fpdb* db);

/* Recommended query row pitch for the device call: the smallest odd multiple
 * of 128 bytes >= pir_fp_min_v_stride (0 for NULL).  The scan reads 64 rows
 * at once; at a power-of-two pitch of many MiB they crowd the same HBM
 * channels (2^24 records x 32 elements, Q = 64: 0.27 ms at pitch 2^24, 0.25
 * ms at 2^24 + 128).  The synchronous call stages rows at this pitch. */
uint64_t pir_fp_v_stride(const pir_fpdb* db);

/*
 * Q queries on device buffers, asynchronous on hip_stream.  d_v: q rows of
 * v_stride bytes (a multiple of 16, >= pir_fp_min_v_stride), base 16-byte
 * aligned; d_out: q * L bytes.  1 <= q <= PIR_MAX_BATCH.  Shares the
 * per-stream workspace rules of pir_dpxor_batch_async.
 */
int pir_fp_inner_async(pir_fpdb* db, const void* d_v, uint64_t v_stride, uint32_t q, void* d_out,
                       void* hip_stream);

/* Q queries, host in and out, synchronous: v holds q rows v_stride >= N
 * bytes apart, out receives q rows of L bytes.  As for pir_dpxor_batch,
 * pinned buffers (pir_host_alloc) are copied to and from the device
 * directly; pageable rows go through two pinned staging pieces of at most
 * 16 MiB each, whatever q is. */
int pir_fp_inner(pir_fpdb* db, const uint8_t* v, uint64_t v_stride, uint32_t q, uint8_t* out);

/* ---------------------------------------------------------------- measurement */

/*
 * Streaming-read probe: the practical HBM read roof that the scans are
 * measured against.  Reads every 16-byte chunk of d_src[0, bytes) once with
 * non-temporal loads, `workgroups` workgroups each taking a contiguous range
 * (unroll = 4, 8 or 16 loads in flight per lane), and writes the XOR of each
 * workgroup's chunks to d_sink, one 16-byte word per workgroup launched.
 * With C = bytes / 16 chunks, a workgroup takes P = ceil(C / workgroups)
 * chunks and ceil(C / P) <= workgroups workgroups run; d_sink holds at least
 * 16 * workgroups bytes and words past the launched ones are not written.
 * The XOR of the written words is the XOR of all chunks.  Asynchronous on hip_stream; device buffers, 16-byte aligned; bytes
 * a positive multiple of 16; 1 <= workgroups <= 2^20.  Errors: PIR_E_INVAL,
 * PIR_E_DEVICE.
 */
int pir_read_probe_async(pir_ctx* ctx, const void* d_src, uint64_t bytes, uint32_t unroll, uint32_t workgroups,
                         void* d_sink, void* hip_stream);

/* ---------------------------------------------------------------- memory */

/* Pinned host memory (hipHostMalloc); NULL on failure.  The synchronous
 * calls copy pinned selection and answer buffers without staging. */
void* pir_host_alloc(size_t bytes);
void pir_host_free(void* p);

#ifdef __cplusplus
}
#endif

#endif /* PIR_H */
