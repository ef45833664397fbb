// Continuous-batching server over resident databases.
//
// The paper's batching scheme (IM-PIR Sec. 3.4, "Batching client queries")
// puts expanded queries on a shared task queue and has scheduler threads hand
// them to DPU clusters as clusters free up.  Here:
//  - each database has its own queue, held in a pinned host ring of selection
//    rows (pir_serve_submit copies the caller's bits straight into the ring,
//    so a batch uploads with one or two host-to-device copies and no extra
//    host copy);
//  - a slot is the GPU analogue of a cluster: a stream with its own device
//    selection, answer and scratch buffers; slots run concurrently;
//  - one scheduler thread retires finished slots (answers to the callers'
//    buffers, latency recorded) and fills free slots with up to q_max pending
//    requests of the database whose oldest request has waited longest.
//    Requests arriving while batches run join the next batches.
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

struct Ticket {
    int status = PIR_OK;
    bool done = false;
};

struct Pending {
    uint64_t ticket;
    uint64_t row;  // absolute ring row index
    uint8_t* out;
    Clock::time_point t_submit;
};

struct DbQueue {
    Db* db = nullptr;
    uint64_t dstride = 0;   // device/ring row pitch (bytes)
    uint64_t row_bytes = 0; // ceil(N/8)
    HostBuf ring;
    uint64_t ring_rows = 0;
    uint64_t next_row = 0;      // next row to fill (absolute)
    uint64_t released_row = 0;  // rows below this are free again (absolute)
    std::deque<Pending> q;
    // batches in flight, in dispatch order: [first_row, end_row, done]
    struct Span { uint64_t first, end; bool done; };
    std::deque<Span> spans;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool busy = false;
    uint32_t db = 0;
    uint64_t span_first = 0;
    std::vector<Pending> reqs;
    HostBuf h_out;
    DevBuf d_sel, d_out, partials;
};

struct Server {
    Ctx* ctx = nullptr;
    pir_serve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
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
    uint64_t hist[13] = {0};
    uint32_t max_inflight = 0;
    Clock::time_point t0;

    void run();
    bool dispatch_one(Slot& s);
    void retire(Slot& s, int status);
};

static uint64_t ring_free(const DbQueue& d) { return d.ring_rows - (d.next_row - d.released_row); }

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
    for (auto& sp : d.spans)
        if (sp.first == s.span_first) sp.done = true;
    while (!d.spans.empty() && d.spans.front().done) {
        d.released_row = d.spans.front().end;
        d.spans.pop_front();
    }
    s.reqs.clear();
    s.busy = false;
}

// Pick the database whose head request is oldest and launch up to q_max of
// its requests on slot s.  Returns false if nothing is ready.
bool Server::dispatch_one(Slot& s) {
    int best = -1;
    Clock::time_point best_t{};
    const auto now = Clock::now();
    for (size_t i = 0; i < dbs.size(); ++i) {
        DbQueue& d = *dbs[i];
        if (d.q.empty()) continue;
        const bool full = d.q.size() >= cfg.q_max;
        const double age_us = std::chrono::duration<double, std::micro>(now - d.q.front().t_submit).count();
        if (!full && !stopping && cfg.max_wait_us && age_us < cfg.max_wait_us) continue;
        if (best < 0 || d.q.front().t_submit < best_t) {
            best = (int)i;
            best_t = d.q.front().t_submit;
        }
    }
    if (best < 0) return false;
    DbQueue& d = *dbs[best];
    const Geometry& g = d.db->geo;
    const uint32_t n = (uint32_t)std::min<size_t>(d.q.size(), cfg.q_max);
    s.reqs.assign(d.q.begin(), d.q.begin() + n);
    d.q.erase(d.q.begin(), d.q.begin() + n);
    s.db = (uint32_t)best;
    s.span_first = s.reqs.front().row;
    d.spans.push_back({s.reqs.front().row, s.reqs.back().row + 1, false});
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
            (e = s.partials.ensure(partial_bytes(g, p, n))) != hipSuccess)
            rc = hip_fail(e, "serving slot buffers");
    }
    // upload the batch's ring rows (contiguous modulo the ring size)
    const uint64_t first = s.reqs.front().row;
    uint64_t done_rows = 0;
    while (rc == PIR_OK && done_rows < n) {
        const uint64_t r = (first + done_rows) % d.ring_rows;
        const uint64_t k = std::min<uint64_t>(n - done_rows, d.ring_rows - r);
        e = hipMemcpyAsync((uint8_t*)s.d_sel.ptr + done_rows * d.dstride, (uint8_t*)d.ring.ptr + r * d.dstride,
                           k * d.dstride, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) rc = hip_fail(e, "selection upload");
        done_rows += k;
    }
    if (rc == PIR_OK) {
        h2d_bytes += (uint64_t)n * d.dstride;
        rc = ctx->enqueue_scan(*d.db, p, (const uint32_t*)s.d_sel.ptr, d.dstride / 4, n, (uint8_t*)s.d_out.ptr,
                               (uint8_t*)s.partials.ptr, s.stream);
    }
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

void Server::run() {
    (void)ctx->bind();
    std::unique_lock<std::mutex> lk(mu);
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
        bool waiting_batches = false;
        for (auto& sp : slots) {
            Slot& s = *sp;
            if (s.busy) continue;
            if (!dispatch_one(s)) break;
            any_busy = any_busy || s.busy;
        }
        for (auto& d : dbs)
            if (!d->q.empty()) waiting_batches = true;
        if (stopping && !waiting_batches && !any_busy) break;
        if (any_busy || waiting_batches) {
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
    raw->th = std::thread([raw] { raw->run(); });
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
    // slot buffers this database may need: selections, answers, scratch
    Plan p;
    int rc = srv->ctx->plan_for(*db, srv->cfg.q_max, nullptr, p);
    if (rc) return rc;
    const uint64_t slot_bytes = dq->dstride * srv->cfg.q_max + (uint64_t)g.R * srv->cfg.q_max +
                                partial_bytes(g, p, srv->cfg.q_max);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) return fail(PIR_E_SHUTDOWN, "server is shutting down");
    const uint64_t need = g.bytes() + slot_bytes * srv->cfg.n_slots;
    if (srv->cfg.hbm_budget_bytes && srv->admitted_bytes + need > srv->cfg.hbm_budget_bytes)
        return fail(PIR_E_NOMEM, "admitting this database needs %llu bytes; %llu of the %llu-byte budget are taken",
                    (unsigned long long)need, (unsigned long long)srv->admitted_bytes,
                    (unsigned long long)srv->cfg.hbm_budget_bytes);
    // pinned request ring: up to 256 MiB, at least 2 batches, at most queue_cap rows
    uint64_t rows = std::max<uint64_t>(2ull * srv->cfg.q_max, (256ull << 20) / dq->dstride);
    rows = std::min<uint64_t>(rows, std::max<uint64_t>(srv->cfg.queue_cap, srv->cfg.q_max));
    hipError_t e = dq->ring.ensure(rows * dq->dstride);
    if (e != hipSuccess) return hip_fail(e, "pinned request ring");
    memset(dq->ring.ptr, 0, rows * dq->dstride);
    dq->ring_rows = rows;
    srv->admitted_bytes += need;
    *db_id = (uint32_t)srv->dbs.size();
    srv->dbs.push_back(std::move(dq));
    return PIR_OK;
}

int pir_serve_submit(pir_server* sv, uint32_t db_id, const uint8_t* sel_bits, uint8_t* out, uint64_t* ticket) {
    clear_error();
    if (!sv || !sel_bits || !out || !ticket) return fail(PIR_E_INVAL, "pir_serve_submit: NULL argument");
    Server* srv = reinterpret_cast<Server*>(sv);
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->stopping) {
        ++srv->rejected;
        return fail(PIR_E_SHUTDOWN, "server is shutting down");
    }
    if (srv->failed) return fail(PIR_E_DEVICE, "server stopped after a device error");
    if (db_id >= srv->dbs.size()) return fail(PIR_E_NOTFOUND, "unknown database id %u", db_id);
    DbQueue& d = *srv->dbs[db_id];
    if (d.q.size() >= srv->cfg.queue_cap || ring_free(d) == 0) {
        ++srv->rejected;
        return fail(PIR_E_BUSY, "queue of database %u is full", db_id);
    }
    const uint64_t row = d.next_row++;
    uint8_t* dst = (uint8_t*)d.ring.ptr + (row % d.ring_rows) * d.dstride;
    memcpy(dst, sel_bits, d.row_bytes);
    const uint64_t t = srv->next_ticket++;
    srv->tickets[t] = Ticket{};
    d.q.push_back({t, row, out, Clock::now()});
    ++srv->submitted;
    *ticket = t;
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
