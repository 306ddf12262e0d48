// Batched and served forms of Algorithm 1 over one resident data graph.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "runtime.hpp"

using namespace dm;

extern "C" dm_status dm_enumerate_batch(dm_datagraph* dg, int32_t n, const dm_graph_desc* gps, const int64_t* caps,
                                        const dm_plan_opts* opts, dm_result** outs) {
    if (!dg || n < 0 || (n > 0 && (!gps || !outs))) return fail(DM_ERR_INVALID_ARG, "invalid batch arguments");
    DM_HIP(hipSetDevice(dg->ctx->device));
    for (int32_t i = 0; i < n; i++) outs[i] = nullptr;
    for (int32_t i = 0; i < n; i++) {
        dm_status st = enumerate_one(dg, dg->ctx->ws, &gps[i], caps ? caps[i] : -1, opts, &outs[i]);
        if (st != DM_OK) {
            for (int32_t j = 0; j < i; j++) dm_result_free(outs[j]), outs[j] = nullptr;
            return st;
        }
    }
    return DM_OK;
}

// ------------------------------------------------------------------ server

namespace {

struct Request {
    uint64_t ticket = 0;
    int32_t nv = 0;
    std::vector<int32_t> edges;
    int64_t cap = -1;
    int64_t est_bytes = 0;
    bool done = false;
    dm_status status = DM_OK;
    std::string err;
    dm_result* result = nullptr;
};

}  // namespace

struct dm_server {
    dm_datagraph* dg = nullptr;
    dm_server_opts opts{};
    std::vector<std::unique_ptr<Workspace>> ws;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
    uint64_t next_ticket = 1;
    int64_t inflight_bytes = 0;
    int32_t inflight = 0;
    bool stopping = false;
};

static void server_worker(dm_server* s, int w) {
    (void)hipSetDevice(s->dg->ctx->device);
    Workspace& ws = *s->ws[w];
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty() && s->stopping) return;
            // admit from the head while the predicted memory fits (always admit one)
            while (!s->queue.empty() && (int32_t)batch.size() < s->opts.max_batch) {
                auto& r = s->queue.front();
                if (!batch.empty() || s->inflight > 0) {
                    if (s->inflight_bytes + r->est_bytes > s->opts.mem_budget) break;
                }
                s->inflight_bytes += r->est_bytes;
                s->inflight++;
                batch.push_back(r);
                s->queue.pop_front();
            }
        }
        for (auto& r : batch) {
            dm_graph_desc gp{r->nv, (int64_t)(r->edges.size() / 2), r->edges.data()};
            dm_result* res = nullptr;
            dm_status st = enumerate_one(s->dg, ws, &gp, r->cap, nullptr, &res);
            std::string err = st == DM_OK ? std::string() : std::string(dm_last_error());
            // the worker synchronized its stream, so the table is complete; later
            // copies and the free are ordered on the context stream, which
            // outlives the server's own streams
            if (res) res->stream = s->dg->ctx->stream;
            std::lock_guard<std::mutex> lk(s->mu);
            r->status = st;
            r->err = err;
            r->result = res;
            r->done = true;
            s->inflight_bytes -= r->est_bytes;
            s->inflight--;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

extern "C" {

dm_status dm_server_start(dm_datagraph* dg, const dm_server_opts* opts, dm_server** out) {
    if (!dg || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    DM_HIP(hipSetDevice(dg->ctx->device));
    auto* s = new dm_server();
    s->dg = dg;
    dm_server_opts o{};
    if (opts) o = *opts;
    if (o.n_streams <= 0) o.n_streams = 2;
    if (o.n_streams > 8) o.n_streams = 8;
    if (o.max_batch <= 0) o.max_batch = 64;
    if (o.mem_budget <= 0) o.mem_budget = (int64_t)8 << 30;
    if (o.max_queue <= 0) o.max_queue = 65536;
    s->opts = o;
    for (int i = 0; i < o.n_streams; i++) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(DM_ERR_DEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
        auto w = std::make_unique<Workspace>();
        dm_status e = w->init(st);
        if (e != DM_OK) {
            w->release();
            for (auto& x : s->ws) x->release();
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return e;
        }
        s->ws.push_back(std::move(w));
    }
    for (int i = 0; i < o.n_streams; i++) s->workers.emplace_back(server_worker, s, i);
    *out = s;
    return DM_OK;
}

dm_status dm_server_submit(dm_server* s, const dm_graph_desc* gp, int64_t max_embeddings, uint64_t* ticket) {
    if (!s || !gp || !ticket) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    NormPattern p;
    std::string err;
    dm_status st = normalize_pattern(gp, &p, &err);
    if (st != DM_OK) return fail(st, err);
    auto r = std::make_shared<Request>();
    r->nv = gp->n_vertices;
    r->edges.assign(gp->edges, gp->edges + 2 * gp->n_edges);
    r->cap = max_embeddings;
    int64_t peak = 0, rows = 0;
    if (dm_estimate(s->dg, gp, nullptr, &peak, &rows) == DM_OK) r->est_bytes = std::max<int64_t>(peak, 1);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(DM_ERR_CANCELLED, "server is stopping");
    if ((int32_t)s->queue.size() >= s->opts.max_queue) return fail(DM_ERR_BUSY, "server queue is full");
    r->ticket = s->next_ticket++;
    s->live[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return DM_OK;
}

dm_status dm_server_wait(dm_server* s, uint64_t ticket, int32_t timeout_ms, dm_result** out) {
    if (!s || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return fail(DM_ERR_INVALID_ARG, "unknown ticket");
    auto r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return fail(DM_ERR_TIMEOUT, "request not finished");
    }
    s->live.erase(ticket);
    if (r->status != DM_OK) return fail(r->status, r->err);
    *out = r->result;
    return DM_OK;
}

dm_status dm_server_stop(dm_server* s) {
    if (!s) return fail(DM_ERR_INVALID_ARG, "NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->live)
        if (kv.second->result) dm_result_free(kv.second->result);
    s->live.clear();
    for (auto& w : s->ws) w->release();
    for (auto x : s->streams) (void)hipStreamDestroy(x);
    delete s;
    return DM_OK;
}

}  // extern "C"
