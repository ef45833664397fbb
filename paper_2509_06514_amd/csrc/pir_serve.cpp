// Continuous-batching server over resident databases.
//
// The paper's batching scheme (IM-PIR Sec. 3.4, "Batching client queries")
// puts expanded queries on a shared task queue and has scheduler threads hand
// them to DPU clusters as clusters free up.  Here:
//  - each database has its own queues, held in pinned host rings: one of
//    selection rows (pir_serve_submit copies the caller's bits straight into
//    the ring, so a batch uploads with one or two host-to-device copies and
//    no extra host copy) and one of DPF keys (pir_serve_submit_key; the
//    server evaluates them, Sec. 3.2, so a query crosses PCIe as a key of
//    64 (n+1) bytes instead of N/8 bytes of bits);
//  - a slot is the GPU analogue of a cluster: a stream with its own device
//    selection, key, answer and scratch buffers; slots run concurrently;
//  - one scheduler thread retires finished slots (answers to the callers'
//    buffers, latency recorded) and fills free slots with up to q_max pending
//    requests of one kind of the database whose oldest request has waited
//    longest.  Requests arriving while batches run join the next batches;
//  - record updates (pir_serve_update) are barriers in a database's request
//    order: an update is applied in an idle window of its database, once
//    every request submitted before it has completed and before any request
//    submitted after it is dispatched, so every answer comes from one whole
//    version of the records (the idle-window updates of Sec. 3.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pir_internal.h"
#include "pir_runtime.h"

namespace pir {

using Clock = std::chrono::steady_clock;

enum Kind { kSel = 0, kKey = 1 };

struct Ticket {
    int status = PIR_OK;
    bool done = false;
};

struct Pending {
    uint64_t ticket;
    uint64_t seq;  // position in the database's submission order (updates included)
    uint64_t row;  // absolute ring row index
    uint8_t* out;
    Clock::time_point t_submit;
};

// Pinned host ring of fixed-size rows; a row is free again once every batch
// up to and including it has retired.
struct Ring {
    HostBuf buf;
    uint64_t stride = 0, rows = 0;
    uint64_t next_row = 0;      // next row to fill (absolute)
    uint64_t released_row = 0;  // rows below this are free again (absolute)
    struct Span { uint64_t first, end; bool done; };
    std::deque<Span> spans;     // batches in flight, in dispatch order

    uint64_t free_rows() const { return rows - (next_row - released_row); }
    uint8_t* row_ptr(uint64_t r) const { return (uint8_t*)buf.ptr + (r % rows) * stride; }
    void finish(uint64_t first) {
        for (auto& sp : spans)
            if (sp.first == first) sp.done = true;
        while (!spans.empty() && spans.front().done) {
            released_row = spans.front().end;
            spans.pop_front();
        }
    }
};

struct UpdateReq {
    uint64_t ticket, seq, first, count;
    std::vector<uint8_t> records;
};

struct DbQueue {
    Db* db = nullptr;
    uint64_t dstride = 0;    // device selection row pitch (bytes)
    uint64_t row_bytes = 0;  // ceil(N/8)
    uint32_t n_bits = 0;     // DPF domain 2^n_bits
    uint64_t key_bytes = 0;
    Ring ring[2];            // kSel: selection rows (pitch dstride); kKey: keys
    std::deque<Pending> q[2];
    std::deque<UpdateReq> updates;
    uint64_t next_seq = 0;
    uint32_t inflight = 0;   // busy slots on this database

    uint64_t barrier() const { return updates.empty() ? UINT64_MAX : updates.front().seq; }
    // requests of kind k that may run before the next update, up to `cap`
    uint32_t eligible(int k, uint32_t cap) const {
        const uint64_t b = barrier();
        uint32_t n = 0;
        for (const Pending& r : q[k]) {
            if (r.seq >= b || n == cap) break;
            ++n;
        }
        return n;
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool busy = false;
    uint32_t db = 0;
    int kind = kSel;
    uint64_t span_first = 0;
    std::vector<Pending> reqs;
    HostBuf h_out;
    DevBuf d_sel, d_out, partials, d_keys;
};

struct Server {
    Ctx* ctx = nullptr;
    pir_serve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::condition_variable cv_ring;  // a batch retired: ring rows may be free again
    std::vector<std::unique_ptr<DbQueue>> dbs;
    std::vector<std::unique_ptr<Slot>> slots;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    uint64_t admitted_bytes = 0;
    bool stopping = false;
    bool failed = false;
    std::thread th;
    // statistics
    std::vector<double> lat_us;
    uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, h2d_bytes = 0;
    uint64_t key_requests = 0, updates_applied = 0, blocked_submits = 0;
    uint64_t hist[13] = {0};
    uint32_t max_inflight = 0;
    Clock::time_point t0;

    void run(std::unique_lock<std::mutex>& lk);
    bool dispatch_one(Slot& s);
    void retire(Slot& s, int status);
    bool apply_ready_update(std::unique_lock<std::mutex>& lk);
    uint64_t new_ticket() {
        const uint64_t t = next_ticket++;
        tickets[t] = Ticket{};
        return t;
    }
};

void Server::retire(Slot& s, int status) {
    DbQueue& d = *dbs[s.db];
    const auto now = Clock::now();
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        const Pending& r = s.reqs[i];
        if (status == PIR_OK) memcpy(r.out, (uint8_t*)s.h_out.ptr + i * d.db->geo.R, d.db->geo.R);
        auto it = tickets.find(r.ticket);
        if (it != tickets.end()) {
            it->second.status = status;
            it->second.done = true;
        }
        lat_us.push_back(std::chrono::duration<double, std::micro>(now - r.t_submit).count());
        ++completed;
    }
    d.ring[s.kind].finish(s.span_first);
    --d.inflight;
    s.reqs.clear();
    s.busy = false;
    cv_ring.notify_all();
}

// Upload ring rows [first, first + n) to dst (contiguous modulo the ring size).
static int upload_rows(const Ring& ring, uint64_t first, uint64_t n, void* dst, hipStream_t s) {
    uint64_t done = 0;
    while (done < n) {
        const uint64_t r = (first + done) % ring.rows;
        const uint64_t k = std::min<uint64_t>(n - done, ring.rows - r);
        hipError_t e = hipMemcpyAsync((uint8_t*)dst + done * ring.stride, (uint8_t*)ring.buf.ptr + r * ring.stride,
                                      k * ring.stride, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "request upload");
        done += k;
    }
    return PIR_OK;
}

// Pick the (database, kind) whose oldest runnable request has waited longest
// and launch up to q_max of its requests on slot s.  Returns false if nothing
// is ready.
bool Server::dispatch_one(Slot& s) {
    int best = -1, best_k = kSel;
    Clock::time_point best_t{};
    const auto now = Clock::now();
    for (size_t i = 0; i < dbs.size(); ++i) {
        DbQueue& d = *dbs[i];
        for (int k = 0; k < 2; ++k) {
            const uint32_t ready = d.eligible(k, cfg.q_max);
            if (ready == 0) continue;
            const bool full = ready >= cfg.q_max;
            const Pending& head = d.q[k].front();
            const double age_us = std::chrono::duration<double, std::micro>(now - head.t_submit).count();
            // a pending update closes the batch: what precedes it runs now
            const bool closed = !d.updates.empty();
            if (!full && !closed && !stopping && cfg.max_wait_us && age_us < cfg.max_wait_us) continue;
            if (best < 0 || head.t_submit < best_t) {
                best = (int)i;
                best_k = k;
                best_t = head.t_submit;
            }
        }
    }
    if (best < 0) return false;
    DbQueue& d = *dbs[best];
    const Geometry& g = d.db->geo;
    const uint32_t n = d.eligible(best_k, cfg.q_max);
    s.reqs.assign(d.q[best_k].begin(), d.q[best_k].begin() + n);
    d.q[best_k].erase(d.q[best_k].begin(), d.q[best_k].begin() + n);
    s.db = (uint32_t)best;
    s.kind = best_k;
    s.span_first = s.reqs.front().row;
    d.ring[best_k].spans.push_back({s.reqs.front().row, s.reqs.back().row + 1, false});
    ++d.inflight;
    ++batches;
    uint32_t bin = 0;
    while ((2u << bin) <= n && bin < 12) ++bin;
    ++hist[bin];

    Plan p;
    int rc = ctx->plan_for(*d.db, n, nullptr, p);
    hipError_t e = hipSuccess;
    if (rc == PIR_OK) {
        if ((e = s.d_sel.ensure(d.dstride * cfg.q_max)) != hipSuccess ||
            (e = s.d_out.ensure((size_t)g.R * cfg.q_max)) != hipSuccess ||
            (e = s.h_out.ensure((size_t)g.R * cfg.q_max)) != hipSuccess ||
            (e = s.partials.ensure(partial_bytes(g, p, n))) != hipSuccess ||
            (best_k == kKey && (e = s.d_keys.ensure(d.key_bytes * cfg.q_max)) != hipSuccess))
            rc = hip_fail(e, "serving slot buffers");
    }
    const uint64_t first = s.reqs.front().row;
    if (rc == PIR_OK && best_k == kSel) {
        rc = upload_rows(d.ring[kSel], first, n, s.d_sel.ptr, s.stream);
        h2d_bytes += (uint64_t)n * d.dstride;
    } else if (rc == PIR_OK) {
        // keys: upload, then evaluate into the slot's selection rows
        rc = upload_rows(d.ring[kKey], first, n, s.d_keys.ptr, s.stream);
        h2d_bytes += (uint64_t)n * d.key_bytes;
        if (rc == PIR_OK)
            rc = dpf_eval_into(ctx, (const uint8_t*)s.d_keys.ptr, d.n_bits, n, g.n, (uint32_t*)s.d_sel.ptr,
                               d.dstride / 4, s.stream);
    }
    if (rc == PIR_OK)
        rc = ctx->launch_scan(*d.db, p, (const uint32_t*)s.d_sel.ptr, d.dstride / 4, n, (uint8_t*)s.d_out.ptr,
                               (uint8_t*)s.partials.ptr, s.stream);
    if (rc == PIR_OK) {
        e = hipMemcpyAsync(s.h_out.ptr, s.d_out.ptr, (size_t)g.R * n, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.done_ev, s.stream);
        if (e != hipSuccess) rc = hip_fail(e, "answer download");
    }
    if (rc != PIR_OK) {
        failed = true;
        (void)hipStreamSynchronize(s.stream);
        retire(s, rc);
        cv_done.notify_all();
        return true;
    }
    s.busy = true;
    uint32_t inflight = 0;
    for (auto& sp : slots) inflight += sp->busy ? 1 : 0;
    max_inflight = std::max(max_inflight, inflight);
    return true;
}

// Apply the first pending update of a database that has reached its idle
// window (nothing before it queued or in flight).  The lock is released while
// the records are written; only this thread dispatches, so nothing of that
// database starts meanwhile.  Returns true if an update was applied.
bool Server::apply_ready_update(std::unique_lock<std::mutex>& lk) {
    for (auto& dp : dbs) {
        DbQueue& d = *dp;
        if (d.updates.empty() || d.inflight || d.eligible(kSel, 1) || d.eligible(kKey, 1)) continue;
        UpdateReq& u = d.updates.front();
        lk.unlock();
        const int rc = pir_db_update(reinterpret_cast<pir_db*>(d.db), u.first, u.count, u.records.data());
        lk.lock();
        auto it = tickets.find(u.ticket);
        if (it != tickets.end()) {
            it->second.status = rc;
            it->second.done = true;
        }
        if (rc == PIR_OK) ++updates_applied;
        d.updates.pop_front();
        cv_done.notify_all();
        return true;
    }
    return false;
}

void Server::run(std::unique_lock<std::mutex>& lk) {
    (void)ctx->bind();
    for (;;) {
        bool any_busy = false, progressed = false;
        for (auto& sp : slots) {
            Slot& s = *sp;
            if (!s.busy) continue;
            hipError_t e = hipEventQuery(s.done_ev);
            if (e == hipSuccess) {
                retire(s, PIR_OK);
                progressed = true;
            } else if (e != hipErrorNotReady) {
                failed = true;
                retire(s, PIR_E_DEVICE);
                progressed = true;
            } else {
                any_busy = true;
            }
        }
        if (progressed) cv_done.notify_all();
        while (apply_ready_update(lk)) {
        }
        for (auto& sp : slots) {
            Slot& s = *sp;
            if (s.busy) continue;
            if (!dispatch_one(s)) break;
            any_busy = any_busy || s.busy;
        }
        bool waiting = false;
        for (auto& d : dbs)
            if (!d->q[kSel].empty() || !d->q[kKey].empty() || !d->updates.empty()) waiting = true;
        if (stopping && !waiting && !any_busy) break;
        if (any_busy || waiting) {
            // poll slot completion (and max_wait deadlines) at a short interval
            cv_sched.wait_for(lk, std::chrono::microseconds(20));
        } else {
            cv_sched.wait(lk);
        }
    }
    cv_done.notify_all();
}

}  // namespace pir

using namespace pir;

extern "C" {

int pir_serve_create(pir_ctx* c, const pir_serve_config* cfg, pir_server** out) {
    clear_error();
    if (!c || !out) return fail(PIR_E_INVAL, "pir_serve_create: NULL argument");
    *out = nullptr;
    auto srv = std::make_unique<Server>();
    srv->ctx = reinterpret_cast<Ctx*>(c);
    if (cfg) srv->cfg = *cfg;
    if (srv->cfg.q_max == 0) srv->cfg.q_max = 64;
    if (srv->cfg.q_max > PIR_MAX_BATCH) return fail(PIR_E_INVAL, "q_max %u > %u", srv->cfg.q_max, PIR_MAX_BATCH);
    if (srv->cfg.n_slots == 0) srv->cfg.n_slots = 4;
    if (srv->cfg.n_slots > 64) return fail(PIR_E_INVAL, "n_slots %u > 64", srv->cfg.n_slots);
    if (srv->cfg.queue_cap == 0) srv->cfg.queue_cap = 65536;
    if (srv->cfg.submit_wait_ms == 0) srv->cfg.submit_wait_ms = 1000;
    if (srv->cfg.ring_bytes == 0) srv->cfg.ring_bytes = 256ull << 20;
    int rc = srv->ctx->bind();
    if (rc) return rc;
    for (uint32_t i = 0; i < srv->cfg.n_slots; ++i) {
        auto s = std::make_unique<Slot>();
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (auto& t : srv->slots) {
                (void)hipEventDestroy(t->done_ev);
                (void)hipStreamDestroy(t->stream);
            }
            if (s->stream) (void)hipStreamDestroy(s->stream);
            return hip_fail(e, "slot stream");
        }
        srv->slots.push_back(std::move(s));
    }
    srv->t0 = Clock::now();
    Server* raw = srv.get();
    raw->th = std::thread([raw] {
        std::unique_lock<std::mutex> lk(raw->mu);
        raw->run(lk);
    });
    *out = reinterpret_cast<pir_server*>(srv.release());
    return PIR_OK;
}

int pir_serve_add_db(pir_server* sv, pir_db* d, uint32_t* db_id) {
    clear_error();
    if (!sv || !d || !db_id) return fail(PIR_E_INVAL, "pir_serve_add_db: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    Db* db = reinterpret_cast<Db*>(d);
    if (db->ctx != srv->ctx) return fail(PIR_E_INVAL, "database belongs to another context");
    const Geometry& g = db->geo;
    auto dq = std::make_unique<DbQueue>();
    dq->db = db;
    dq->row_bytes = (g.n + 7) / 8;
    dq->dstride = (4ull * g.nb + 255) / 256 * 256;
    dq->n_bits = pir_dpf_domain_bits(g.n);
    dq->key_bytes = dpf_key_bytes(dq->n_bits);
    // slot buffers this database may need: selections, keys, answers, scratch,
    // DPF evaluation scratch
    Plan p;
    int rc = srv->ctx->plan_for(*db, srv->cfg.q_max, nullptr, p);
    if (rc) return rc;
    const uint64_t slot_bytes = dq->dstride * srv->cfg.q_max + dq->key_bytes * srv->cfg.q_max +
                                (uint64_t)g.R * srv->cfg.q_max + partial_bytes(g, p, srv->cfg.q_max) +
                                dpf_eval_scratch_bytes(dq->n_bits, g.n, srv->cfg.q_max);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return fail(PIR_E_SHUTDOWN, "server is shutting down");
    const uint64_t need = g.bytes() + slot_bytes * srv->cfg.n_slots;
    if (srv->cfg.hbm_budget_bytes && srv->admitted_bytes + need > srv->cfg.hbm_budget_bytes)
        return fail(PIR_E_NOMEM, "admitting this database needs %llu bytes; %llu of the %llu-byte budget are taken",
                    (unsigned long long)need, (unsigned long long)srv->admitted_bytes,
                    (unsigned long long)srv->cfg.hbm_budget_bytes);
    // pinned request rings: ring_bytes of selection rows (default 256 MiB)
    // and 16 MiB of keys, but at least one batch per slot plus one queued
    // batch, and no more than can ever be in use (queue_cap queued plus a full
    // batch in every slot)
    const uint64_t cap_rows = (uint64_t)srv->cfg.queue_cap + (uint64_t)srv->cfg.n_slots * srv->cfg.q_max;
    const uint64_t min_rows = (uint64_t)(srv->cfg.n_slots + 1) * srv->cfg.q_max;
    const uint64_t strides[2] = {dq->dstride, dq->key_bytes};
    const uint64_t budgets[2] = {srv->cfg.ring_bytes, 16ull << 20};
    for (int k = 0; k < 2; ++k) {
        uint64_t rows = std::max<uint64_t>(min_rows, budgets[k] / strides[k]);
        rows = std::min<uint64_t>(rows, cap_rows);
        hipError_t e = dq->ring[k].buf.ensure(rows * strides[k]);
        if (e != hipSuccess) return hip_fail(e, "pinned request ring");
        memset(dq->ring[k].buf.ptr, 0, rows * strides[k]);
        dq->ring[k].rows = rows;
        dq->ring[k].stride = strides[k];
    }
    srv->admitted_bytes += need;
    *db_id = (uint32_t)srv->dbs.size();
    srv->dbs.push_back(std::move(dq));
    return PIR_OK;
}

}  // extern "C"

namespace pir {

// Admission of one request of kind k into database db_id's queue (mu held).
// PIR_E_BUSY only when the database's queue holds queue_cap requests; when
// the queue has room but the pinned ring has no free row (every row belongs
// to a queued or in-flight request), the caller waits for a batch to retire,
// at most submit_wait_ms, before PIR_E_BUSY.
static int admit(Server* srv, std::unique_lock<std::mutex>& lk, uint32_t db_id, int k, DbQueue** out) {
    if (srv->stopping) {
        ++srv->rejected;
        return fail(PIR_E_SHUTDOWN, "server is shutting down");
    }
    if (srv->failed) return fail(PIR_E_DEVICE, "server stopped after a device error");
    if (db_id >= srv->dbs.size()) return fail(PIR_E_NOTFOUND, "unknown database id %u", db_id);
    DbQueue& d = *srv->dbs[db_id];
    if (d.q[k].size() >= srv->cfg.queue_cap) {
        ++srv->rejected;
        return fail(PIR_E_BUSY, "%s queue of database %u holds queue_cap = %u requests", k == kSel ? "selection" : "key",
                    db_id, srv->cfg.queue_cap);
    }
    if (d.ring[k].free_rows() == 0) {
        ++srv->blocked_submits;
        const auto until = Clock::now() + std::chrono::milliseconds(srv->cfg.submit_wait_ms);
        srv->cv_ring.wait_until(lk, until, [&] { return d.ring[k].free_rows() > 0 || srv->stopping || srv->failed; });
        if (srv->stopping) {
            ++srv->rejected;
            return fail(PIR_E_SHUTDOWN, "server is shutting down");
        }
        if (srv->failed) return fail(PIR_E_DEVICE, "server stopped after a device error");
        if (d.ring[k].free_rows() == 0) {
            ++srv->rejected;
            return fail(PIR_E_BUSY, "no pinned ring row of database %u freed within %u ms", db_id,
                        srv->cfg.submit_wait_ms);
        }
        if (d.q[k].size() >= srv->cfg.queue_cap) {
            ++srv->rejected;
            return fail(PIR_E_BUSY, "queue of database %u holds queue_cap = %u requests", db_id, srv->cfg.queue_cap);
        }
    }
    *out = &d;
    return PIR_OK;
}

}  // namespace pir

extern "C" {

int pir_serve_submit(pir_server* sv, uint32_t db_id, const uint8_t* sel_bits, uint8_t* out, uint64_t* ticket) {
    clear_error();
    if (!sv || !sel_bits || !out || !ticket) return fail(PIR_E_INVAL, "pir_serve_submit: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::unique_lock<std::mutex> lk(srv->mu);
    DbQueue* dp = nullptr;
    const int rc = admit(srv, lk, db_id, kSel, &dp);
    if (rc) return rc;
    DbQueue& d = *dp;
    const uint64_t row = d.ring[kSel].next_row++;
    memcpy(d.ring[kSel].row_ptr(row), sel_bits, d.row_bytes);
    const uint64_t t = srv->new_ticket();
    d.q[kSel].push_back({t, d.next_seq++, row, out, Clock::now()});
    ++srv->submitted;
    *ticket = t;
    lk.unlock();
    srv->cv_sched.notify_one();
    return PIR_OK;
}

int pir_serve_submit_key(pir_server* sv, uint32_t db_id, const uint8_t* key, uint8_t* out, uint64_t* ticket) {
    clear_error();
    if (!sv || !key || !out || !ticket) return fail(PIR_E_INVAL, "pir_serve_submit_key: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::unique_lock<std::mutex> lk(srv->mu);
    DbQueue* dp = nullptr;
    const int rc = admit(srv, lk, db_id, kKey, &dp);
    if (rc) return rc;
    DbQueue& d = *dp;
    const uint64_t row = d.ring[kKey].next_row++;
    memcpy(d.ring[kKey].row_ptr(row), key, d.key_bytes);
    const uint64_t t = srv->new_ticket();
    d.q[kKey].push_back({t, d.next_seq++, row, out, Clock::now()});
    ++srv->submitted;
    ++srv->key_requests;
    *ticket = t;
    lk.unlock();
    srv->cv_sched.notify_one();
    return PIR_OK;
}

int pir_serve_update(pir_server* sv, uint32_t db_id, uint64_t first, uint64_t count, const void* records,
                     uint64_t* ticket) {
    clear_error();
    if (!sv || !records || !ticket) return fail(PIR_E_INVAL, "pir_serve_update: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->stopping) return fail(PIR_E_SHUTDOWN, "server is shutting down");
    if (srv->failed) return fail(PIR_E_DEVICE, "server stopped after a device error");
    if (db_id >= srv->dbs.size()) return fail(PIR_E_NOTFOUND, "unknown database id %u", db_id);
    DbQueue& d = *srv->dbs[db_id];
    const Geometry& g = d.db->geo;
    if (count == 0 || first >= g.n || count > g.n - first)
        return fail(PIR_E_INVAL, "pir_serve_update: range [%llu, +%llu) outside N=%llu", (unsigned long long)first,
                    (unsigned long long)count, (unsigned long long)g.n);
    UpdateReq u;
    u.first = first;
    u.count = count;
    u.records.assign((const uint8_t*)records, (const uint8_t*)records + count * g.R);
    u.ticket = srv->new_ticket();
    u.seq = d.next_seq++;
    *ticket = u.ticket;
    d.updates.push_back(std::move(u));
    lk.unlock();
    srv->cv_sched.notify_one();
    return PIR_OK;
}

int pir_serve_wait(pir_server* sv, uint64_t ticket, int timeout_ms) {
    clear_error();
    if (!sv) return fail(PIR_E_INVAL, "pir_serve_wait: NULL server");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(PIR_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    auto done = [&] { return srv->tickets[ticket].done; };
    if (timeout_ms < 0) {
        srv->cv_done.wait(lk, done);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        return fail(PIR_E_TIMEOUT, "ticket %llu still pending", (unsigned long long)ticket);
    }
    const int st = srv->tickets[ticket].status;
    srv->tickets.erase(ticket);
    if (st != PIR_OK) return fail(st, "request failed");
    return PIR_OK;
}

int pir_serve_poll(pir_server* sv, uint64_t ticket, int* status) {
    clear_error();
    if (!sv || !status) return fail(PIR_E_INVAL, "pir_serve_poll: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(PIR_E_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return 0;
    *status = it->second.status;
    srv->tickets.erase(it);
    return 1;
}

int pir_serve_stats_get(pir_server* sv, pir_serve_stats* out, int reset) {
    clear_error();
    if (!sv || !out) return fail(PIR_E_INVAL, "pir_serve_stats_get: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::lock_guard<std::mutex> lk(srv->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->batches = srv->batches;
    out->h2d_bytes = srv->h2d_bytes;
    for (int i = 0; i < 13; ++i) out->batch_hist[i] = srv->hist[i];
    out->max_inflight = srv->max_inflight;
    out->n_slots = (uint32_t)srv->slots.size();
    out->key_requests = srv->key_requests;
    out->updates_applied = srv->updates_applied;
    out->blocked_submits = srv->blocked_submits;
    out->elapsed_s = std::chrono::duration<double>(Clock::now() - srv->t0).count();
    out->qps = out->elapsed_s > 0 ? (double)srv->completed / out->elapsed_s : 0.0;
    if (!srv->lat_us.empty()) {
        std::vector<double> v(srv->lat_us);
        auto pct = [&](double f) {
            size_t k = (size_t)std::min<double>(v.size() - 1, std::floor(f * (v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return v[k];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        double sum = 0, mx = 0;
        for (double x : srv->lat_us) {
            sum += x;
            mx = std::max(mx, x);
        }
        out->mean_us = sum / srv->lat_us.size();
        out->max_us = mx;
    }
    if (reset) {
        srv->lat_us.clear();
        srv->submitted = srv->completed = srv->rejected = srv->batches = srv->h2d_bytes = 0;
        srv->key_requests = srv->updates_applied = srv->blocked_submits = 0;
        for (auto& h : srv->hist) h = 0;
        srv->max_inflight = 0;
        srv->t0 = Clock::now();
    }
    return PIR_OK;
}

int pir_serve_destroy(pir_server* sv) {
    clear_error();
    if (!sv) return fail(PIR_E_INVAL, "pir_serve_destroy: NULL");
    Server* srv = reinterpret_cast<Server*>(sv);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_sched.notify_all();
    srv->cv_ring.notify_all();
    if (srv->th.joinable()) srv->th.join();
    (void)srv->ctx->bind();
    for (auto& s : srv->slots) {
        if (s->stream) (void)hipStreamSynchronize(s->stream);
        if (s->done_ev) (void)hipEventDestroy(s->done_ev);
        if (s->stream) (void)hipStreamDestroy(s->stream);
    }
    srv->slots.clear();
    srv->dbs.clear();
    delete srv;
    return PIR_OK;
}

}  // extern "C"
