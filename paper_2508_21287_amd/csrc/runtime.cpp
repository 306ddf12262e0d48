// Host runtime: contexts, the resident data graph (Algorithm 2), the plan
// executor (Algorithm 1) and the C ABI entry points of libdmotif.so.
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <functional>

namespace dm {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
dm_status fail(dm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}
dm_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? DM_ERR_OUT_OF_MEMORY : DM_ERR_DEVICE;
}

// Return every cached block to the pool (on the context's stream).
static void flush_blocks(const dm_context* ctx) {
    BlockCache& bc = ctx->blocks;
    std::lock_guard<std::mutex> lk(bc.mu);
    for (auto& b : bc.bins)
        for (void* q : b.second) (void)hipFreeAsync(q, ctx->stream);
    bc.bins.clear();
    bc.cached = 0;
}

dm_status dev_alloc(const dm_context* ctx, void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (ctx && ctx->has_alloc) {
        *p = ctx->alloc.alloc(bytes, (void*)s, ctx->alloc.user);
        if (!*p) return fail(DM_ERR_OUT_OF_MEMORY, "the context's allocator returned NULL for " +
                                                       std::to_string(bytes) + " bytes");
        return DM_OK;
    }
    const bool cacheable = ctx && bytes <= BlockCache::kMaxBlock;
    if (cacheable) {
        BlockCache& bc = ctx->blocks;
        const size_t cls = BlockCache::size_class(bytes);
        {
            std::lock_guard<std::mutex> lk(bc.mu);
            auto it = bc.bins.find(cls);
            if (it != bc.bins.end() && !it->second.empty()) {
                bool ok = true;
                if (s != ctx->stream) {
                    // the block was freed in the context stream's order: this
                    // stream waits for everything enqueued there so far
                    if (!bc.ev) ok = hipEventCreateWithFlags(&bc.ev, hipEventDisableTiming) == hipSuccess;
                    ok = ok && hipEventRecord(bc.ev, ctx->stream) == hipSuccess &&
                         hipStreamWaitEvent(s, bc.ev, 0) == hipSuccess;
                    if (!ok) (void)hipGetLastError();
                }
                if (ok) {
                    *p = it->second.back();
                    it->second.pop_back();
                    bc.cached -= cls;
                    bc.live[*p] = cls;
                    return DM_OK;
                }
            }
        }
        hipError_t e = hipMallocAsync(p, cls, s);
        if (e != hipSuccess) {
            // the cache may hold what the pool lacks: give it back and retry once
            (void)hipGetLastError();
            flush_blocks(ctx);
            e = hipMallocAsync(p, cls, s);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return hip_fail(e, "hipMallocAsync");
        }
        std::lock_guard<std::mutex> lk(bc.mu);
        bc.live[*p] = cls;
        return DM_OK;
    }
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e != hipSuccess && ctx) {
        (void)hipGetLastError();
        flush_blocks(ctx);
        e = hipMallocAsync(p, bytes, s);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return hip_fail(e, "hipMallocAsync");
    }
    return DM_OK;
}

void dev_free(const dm_context* ctx, void* p, hipStream_t s) {
    if (!p) return;
    if (ctx && ctx->has_alloc) {
        ctx->alloc.free(p, (void*)s, ctx->alloc.user);
        return;
    }
    if (ctx) {
        BlockCache& bc = ctx->blocks;
        std::lock_guard<std::mutex> lk(bc.mu);
        auto it = bc.live.find(p);
        if (it != bc.live.end()) {
            const size_t cls = it->second;
            bc.live.erase(it);
            // kept for reuse only when freed in the order of the context's stream
            if (s == ctx->stream && bc.cached + cls <= BlockCache::kMaxCached) {
                bc.bins[cls].push_back(p);
                bc.cached += cls;
                return;
            }
        }
    }
    (void)hipFreeAsync(p, s);
}

WaitCtl wait_ctl(const dm_context* ctx, uint32_t* abort, WaitDiag* diag, int64_t limit_us) {
    WaitCtl w;
    w.abort = abort;
    w.diag = diag;
    w.cancel = ctx ? ctx->cancel : nullptr;
    const int64_t us = limit_us > 0 ? limit_us : 10000000;  // default: 10 s without progress
    const int64_t khz = ctx && ctx->wall_khz > 0 ? ctx->wall_khz : 100000;
    w.limit = std::max<uint64_t>((uint64_t)us * (uint64_t)khz / 1000, 1);
    return w;
}

dm_status check_abort(uint32_t abort, const WaitDiag& d, const char* where) {
    if (abort == 0) return DM_OK;
    if (abort == WAIT_CANCEL || d.reason == WAIT_CANCEL)
        return fail(DM_ERR_CANCELLED, std::string(where) + ": cancelled (dm_context_cancel)");
    char buf[320];
    if (d.reason == WAIT_IDLE)
        std::snprintf(buf, sizeof buf,
                      "%s: persistent scheduler found no tile finishing for %lld wall-clock ticks (%lld polls); "
                      "first unfinished pattern %d at step %d (%d tiles, %d claimed, %d finished)",
                      where, (long long)d.ticks, (long long)d.spins, d.pattern, d.step, d.ntiles, d.claimed,
                      d.finished);
    else
        std::snprintf(buf, sizeof buf,
                      "%s: look-back of tile %lld (pattern %d, step %d) waited %lld wall-clock ticks (%lld polls) "
                      "for a predecessor",
                      where, (long long)d.tile, d.pattern, d.step, (long long)d.ticks, (long long)d.spins);
    return fail(DM_ERR_DEVICE, buf);
}

// ------------------------------------------------------------- workspace

// A fixed workspace cannot grow: the request does not fit its scratch.
static dm_status fixed_full(const char* what) {
    return fail(DM_ERR_BUDGET_EXCEEDED, std::string(what) + " does not fit the fixed scratch");
}

dm_status Workspace::init(dm_context* c, hipStream_t s) {
    ctx = c;
    stream = s;
    DM_TRY(dev_alloc(ctx, (void**)&tickets, sizeof(uint64_t) * kEpochs, s));
    DM_HIP(launch_fill_u64(tickets, 0, kEpochs, s));
    DM_TRY(dev_alloc(ctx, (void**)&ctrl_d, sizeof(Control), s));
    DM_HIP(hipHostMalloc((void**)&ctrl_h, sizeof(Control), hipHostMallocDefault));
    std::memset(ctrl_h, 0, sizeof(Control));
    DM_HIP(hipEventCreate(&ev[0]));
    DM_HIP(hipEventCreate(&ev[1]));
    DM_TRY(dev_alloc(ctx, (void**)&job_d, sizeof(SortJob), s));
    DM_HIP(hipHostMalloc((void**)&job_h, sizeof(SortJob), hipHostMallocDefault));
    epoch = 0;
    return DM_OK;
}

void Workspace::release() {
    for (int i = 0; i < 2; i++) dev_free(ctx, buf[i], stream), buf[i] = nullptr, buf_elems[i] = 0;
    dev_free(ctx, status, stream);
    dev_free(ctx, tickets, stream);
    dev_free(ctx, ctrl_d, stream);
    dev_free(ctx, spill, stream);
    dev_free(ctx, sort_scratch, stream);
    dev_free(ctx, heap, stream);
    dev_free(ctx, heap_words, stream);
    for (int i = 0; i < 2; i++) dev_free(ctx, cbuf[i], stream), cbuf[i] = nullptr, cbuf_rows[i] = 0;
    heap = nullptr;
    heap_words = nullptr;
    heap_elems = heap_words_cap = 0;
    status = nullptr;
    tickets = nullptr;
    ctrl_d = nullptr;
    spill = nullptr;
    spill_bits = nullptr;
    spill_cap = 0;
    sort_scratch = nullptr;
    if (stream) (void)hipStreamSynchronize(stream);
    if (ctrl_h) (void)hipHostFree(ctrl_h);
    ctrl_h = nullptr;
    dev_free(ctx, job_d, stream);
    job_d = nullptr;
    if (job_h) (void)hipHostFree(job_h);
    job_h = nullptr;
    if (stage_h) (void)hipHostFree(stage_h);
    stage_h = nullptr;
    stage_bytes = 0;
    for (int i = 0; i < 2; i++)
        if (ev[i]) (void)hipEventDestroy(ev[i]), ev[i] = nullptr;
    for (auto e : prof) (void)hipEventDestroy(e);
    prof.clear();
}

// Pinned so that several device-to-host copies can be queued and waited for
// once (a copy into pageable memory waits for the device by itself).  The
// caller synchronizes the stream before the buffer is reused or grown.
dm_status Workspace::ensure_stage(size_t bytes) {
    if (stage_bytes >= bytes) return DM_OK;
    if (fixed) return fixed_full("host staging");
    if (stage_h) {
        if (stream) DM_HIP(hipStreamSynchronize(stream));
        (void)hipHostFree(stage_h);
        stage_h = nullptr;
        stage_bytes = 0;
    }
    const size_t c = std::max<size_t>(bytes, (size_t)1 << 16);
    DM_HIP(hipHostMalloc((void**)&stage_h, c, hipHostMallocDefault));
    stage_bytes = c;
    return DM_OK;
}

dm_status Workspace::ensure_buf(int i, int64_t elems) {
    if (buf_elems[i] >= elems) return DM_OK;
    if (fixed) return fixed_full("an intermediate table");
    dev_free(ctx, buf[i], stream);
    buf[i] = nullptr;
    buf_elems[i] = 0;
    int64_t e = std::max<int64_t>(elems, 1 << 16);
    DM_TRY(dev_alloc(ctx, (void**)&buf[i], sizeof(int32_t) * (size_t)e, stream));
    buf_elems[i] = e;
    return DM_OK;
}

dm_status Workspace::ensure_status(int64_t words) {
    if (status_cap >= words) return DM_OK;
    if (fixed) return fixed_full("the look-back words");
    dev_free(ctx, status, stream);
    status = nullptr;
    int64_t w = std::max<int64_t>(words, 1 << 14);
    DM_TRY(dev_alloc(ctx, (void**)&status, sizeof(uint64_t) * (size_t)w, stream));
    DM_HIP(launch_fill_u64(status, 0, w, stream));
    status_cap = w;
    return DM_OK;
}

dm_status Workspace::ensure_spill(int64_t n) {
    if (spill_cap >= n) return DM_OK;
    if (fixed) return fixed_full("the sort's segment lists");
    dev_free(ctx, spill, stream);
    spill = nullptr;
    spill_bits = nullptr;
    int64_t c = std::max<int64_t>(n, 1024);
    DM_TRY(dev_alloc(ctx, (void**)&spill, sizeof(SegRef) * 2 * (size_t)c + sizeof(uint32_t) * (size_t)c, stream));
    spill_cap = c;
    spill_bits = (uint32_t*)(spill + 2 * c);
    // epoch words: zero is no epoch (epochs start at 1)
    DM_HIP(launch_fill_i32((int32_t*)spill_bits, 0, c, stream));
    return DM_OK;
}

dm_status Workspace::ensure_cbuf(int i, int64_t rows) {
    if (cbuf_rows[i] >= rows) return DM_OK;
    if (fixed) return fixed_full("the layout costs");
    dev_free(ctx, cbuf[i], stream);
    cbuf[i] = nullptr;
    cbuf_rows[i] = 0;
    DM_TRY(dev_alloc(ctx, (void**)&cbuf[i], sizeof(uint64_t) * (size_t)std::max<int64_t>(rows, 1), stream));
    cbuf_rows[i] = rows;
    return DM_OK;
}

dm_status Workspace::ensure_heap(int64_t elems, int64_t min_elems, int64_t min_words) {
    elems = std::max(elems, min_elems);
    int64_t words = std::max<int64_t>(elems / 32 + 65536, min_words);
    if (heap_elems >= elems && heap_words_cap >= words) return DM_OK;
    if (fixed) return fixed_full("the batch heap");
    elems = std::max(elems, heap_elems);
    words = std::max(words, heap_words_cap);
    dev_free(ctx, heap, stream);
    heap = nullptr;
    heap_elems = 0;
    dev_free(ctx, heap_words, stream);
    heap_words = nullptr;
    heap_words_cap = 0;
    DM_TRY(dev_alloc(ctx, (void**)&heap, sizeof(int32_t) * (size_t)elems, stream));
    heap_elems = elems;
    DM_TRY(dev_alloc(ctx, (void**)&heap_words, sizeof(uint64_t) * (size_t)words, stream));
    heap_words_cap = words;
    DM_HIP(launch_fill_u64(heap_words, 0, words, stream));
    heap_epoch = 0;
    return DM_OK;
}

uint32_t Workspace::next_heap_epoch() {
    if (++heap_epoch >= kEpochs) {
        if (launch_fill_u64(heap_words, 0, heap_words_cap, stream) != hipSuccess) return 0;
        heap_epoch = 1;
    }
    return heap_epoch;
}

dm_status Workspace::ensure_sort_scratch(int64_t elems) {
    if (sort_scratch_elems >= elems) return DM_OK;
    if (fixed) return fixed_full("the sort's index scratch");
    dev_free(ctx, sort_scratch, stream);
    sort_scratch = nullptr;
    int64_t c = std::max<int64_t>(elems, 1 << 16);
    DM_TRY(dev_alloc(ctx, (void**)&sort_scratch, sizeof(uint32_t) * (size_t)c, stream));
    sort_scratch_elems = c;
    return DM_OK;
}

dm_status Workspace::next_epoch(uint32_t* e) {
    epoch++;
    if (epoch >= kEpochs) {
        // all epochs used: clear every look-back word, ticket and sort epoch word, start over
        DM_HIP(launch_fill_u64(status, 0, status_cap, stream));
        DM_HIP(launch_fill_u64(tickets, 0, kEpochs, stream));
        if (spill_bits) DM_HIP(launch_fill_i32((int32_t*)spill_bits, 0, spill_cap, stream));
        epoch = 1;
    }
    *e = epoch;
    return DM_OK;
}

// ------------------------------------------------------------- plan execution

static int auto_block(double est_rows) { return est_rows < 65536.0 ? 64 : 256; }

static int ejf_grid(int64_t in_cap, double est_in, int block) {
    int64_t tiles_cap = (in_cap + block - 1) / block;
    int64_t g = (int64_t)std::ceil(2.0 * std::max(est_in, 1.0) / block);
    g = std::max<int64_t>(g, 64);
    g = std::min<int64_t>(g, 2048);
    g = std::min<int64_t>(g, std::max<int64_t>(tiles_cap, 1));
    return (int)std::max<int64_t>(g, 1);
}


dm_status enqueue_sort(dm_context* ctx, Workspace& ws, const SortJob* jobs_d, int32_t n_jobs, int32_t nv,
                       int32_t v0, int64_t max_in_cap, int32_t max_wp, int32_t* counters, const uint32_t* abort,
                       int32_t* host_word, hipEvent_t* prof, bool* merged, int32_t stream_k, bool* merge_later,
                       const SortJob* one) {
    if (merged) *merged = false;
    if (one && (n_jobs != 1 || !merge_later))
        return fail(DM_ERR_INTERNAL, "a sort job passed with the launch takes one table and the deferred merge tier");
    hipStream_t s = ws.stream;
    const int64_t items = (int64_t)n_jobs * nv;
    if (items >= (int64_t)INT32_MAX) return fail(DM_ERR_UNSUPPORTED, "batch too large: patterns x vertices >= 2^31");
    DM_TRY(ws.ensure_spill(items + 1));
    SortLaunch L;
    std::memset(&L, 0, sizeof L);
    L.jobs = one ? nullptr : jobs_d;
    if (one) L.one = *one;
    L.n_jobs = n_jobs;
    L.n_vertices = nv;
    L.v_begin = v0;
    L.dup_count = &counters[3];
    L.max_chunks = &counters[2];
    L.abort = abort;
    // tier 1: small LDS tiles (16 KB: swept on the benchmark against 8-48 KB,
    // more resident workgroups beat holding larger segments here); one
    // workgroup per (job, root) item up to 65536 of them, so the hardware
    // dispatcher, which starts a workgroup as soon as one finishes, balances
    // the very uneven segments
    L.lds_bytes = 16 * 1024 - 512;
    L.list = nullptr;
    L.spill = ws.spill;
    L.spill_n = &counters[0];
    int64_t grid1 = std::min<int64_t>(std::max<int64_t>(items, 1), 65536);
    if (n_jobs == 1 && stream_k > 0) {
        // one table: a streaming pass writes every row in place and marks the
        // root segments out of order with a fresh epoch (no clearing launch);
        // tier 1 visits the marked ones only
        uint32_t ep = 0;
        DM_TRY(ws.next_epoch(&ep));
        L.todo_epoch = ep;
        DM_HIP(launch_sort_stream(L, ws.spill_bits, &counters[4], max_in_cap, stream_k, s));
        L.todo = ws.spill_bits;
    }
    // a table whose root segments average at most 32 rows (the 16-vertex
    // trees on the lattices: ~17) takes one-wave workgroups with 4 KB of
    // LDS, 32 resident per CU instead of 8 (the rare longer segment goes on
    // to tier 2): the per-segment rounds (search, staging, write) overlap
    // (tree tables 0.94 -> 0.57 ms per step; 8 KB: 0.60, 128 threads: 0.69)
    int t1_threads = 256;
    if (n_jobs == 1 && items > 0 && max_in_cap <= 32 * items) {
        t1_threads = 64;
        L.lds_bytes = 4096 - 256;
    }
    DM_HIP(launch_sort_lds(L, (int)grid1, t1_threads, L.lds_bytes, s));
    L.todo = nullptr;
    // tier 2: the largest LDS allocation a workgroup can hold; one such
    // workgroup fills a CU, so it takes the largest block
    L.lds_bytes = ctx->sort_lds_max;
    L.list = ws.spill;
    L.list_n = &counters[0];
    L.spill = ws.spill + ws.spill_cap;
    L.spill_n = &counters[1];
    DM_HIP(launch_sort_lds(L, 256, 1024, L.lds_bytes, s));
    // tier 3: chunks of the tier-2 tile, merged pairwise.  No segment
    // outgrows the tier-2 tile when no table has more rows than it holds;
    // else the number of segments tier 2 passed on decides: read back here,
    // or, with merge_later, by the caller with its own readback (then
    // enqueue_sort_merge runs the tier when there are any).
    if (prof) DM_HIP(hipEventRecord(prof[0], s));
    const int64_t r_min = std::max(lds_rows_of(L.lds_bytes, max_wp), 1);
    if (merge_later) *merge_later = max_in_cap > r_min;
    if (max_in_cap <= r_min || merge_later) return DM_OK;
    DM_HIP(hipMemcpyAsync(host_word, &counters[1], sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    if (*host_word == 0) return DM_OK;
    if (merged) *merged = true;
    return enqueue_sort_merge(ctx, ws, jobs_d, n_jobs, nv, v0, max_in_cap, max_wp, counters, abort,
                              prof ? prof + 1 : nullptr);
}

dm_status enqueue_sort_merge(dm_context* ctx, Workspace& ws, const SortJob* jobs_d, int32_t n_jobs, int32_t nv,
                             int32_t v0, int64_t max_in_cap, int32_t max_wp, int32_t* counters, const uint32_t* abort,
                             hipEvent_t* prof) {
    hipStream_t s = ws.stream;
    SortLaunch L;
    std::memset(&L, 0, sizeof L);
    L.jobs = jobs_d;
    L.n_jobs = n_jobs;
    L.n_vertices = nv;
    L.v_begin = v0;
    L.dup_count = &counters[3];
    L.max_chunks = &counters[2];
    L.abort = abort;
    L.lds_bytes = ctx->sort_lds_max;
    const int64_t r_min = std::max(lds_rows_of(L.lds_bytes, max_wp), 1);
    if (prof) DM_HIP(hipEventRecord(prof[0], s));
    L.list = ws.spill + ws.spill_cap;
    L.list_n = &counters[1];
    const int64_t chunks = (std::max<int64_t>(max_in_cap, 1) + r_min - 1) / r_min;
    int passes = 0;
    while (((int64_t)1 << passes) < chunks) passes++;
    DM_HIP(launch_sort_merge_tier(L, passes, s));
    if (prof) DM_HIP(hipEventRecord(prof[1], s));
    return DM_OK;
}

dm_status run_plan(dm_context* ctx, Workspace& ws, const dm_datagraph* dg, const Plan& plan,
                   const RunOptions& opt, RunOutput* out) {
    (void)ctx;
    hipStream_t s = ws.stream;
    const int k = plan.k;
    const int32_t v0 = opt.root_end > opt.root_begin ? opt.root_begin : 0;
    const int32_t v1 = opt.root_end > opt.root_begin ? opt.root_end : dg->n;
    std::vector<StepDesc> steps;
    std::vector<double> est;
    for (auto& ps : plan.steps) {
        steps.push_back(ps.d);
        est.push_back(ps.est_rows);
    }
    if (steps.empty()) {  // 1-vertex pattern: a no-op filter materializes the identity table
        StepDesc d;
        std::memset(&d, 0, sizeof d);
        d.motif = -1;
        d.c_in = 1;
        steps.push_back(d);
        est.push_back((double)dg->n);
    }
    const int nsteps = (int)steps.size();
    if (nsteps > kMaxSteps) return fail(DM_ERR_UNSUPPORTED, "plan has too many steps");
    const bool hash_mode = opt.mode == DM_OUT_COUNT_HASH;

    // the planner's estimates are for every root; scale them to this range
    const double frac = dg->n > 0 ? (double)(v1 - v0) / dg->n : 1.0;
    double est_max = (double)(v1 - v0);
    for (double& e : est) {
        e *= frac;
        est_max = std::max(est_max, e);
    }
    int64_t budget = opt.mem_budget > 0 ? opt.mem_budget : (int64_t)48 << 30;
    int64_t budget_rows = std::max<int64_t>(budget / (int64_t)(8 * k), 1024);
    // first attempt: twice the estimate, at most 1 GiB per table; a larger
    // real table costs one re-run with exact sizes (sync mode)
    const int64_t first_max = std::min<int64_t>(budget_rows, ((int64_t)1 << 28) / k);
    int64_t cap0 = (int64_t)std::min<double>(est_max * 2.0 + 4096.0, (double)first_max);
    cap0 = std::max<int64_t>(cap0, std::min<int64_t>(1 << 14, budget_rows));
    if (opt.initial_rows > 0) cap0 = std::min<int64_t>(opt.initial_rows, budget_rows);
    // a fixed workspace: its buffers as they are (every table gets all of them)
    if (ws.fixed) cap0 = std::max<int64_t>(std::min(ws.buf_elems[0], ws.buf_elems[1]) / k, 1);
    const int block = opt.block > 0 ? opt.block : auto_block(est_max);

    // capacity (rows) of each ping-pong buffer; stride of a table = its capacity
    int64_t cap[2] = {cap0, cap0};
    bool sync_mode = opt.sync_each_step;
    RunOutput o;
    int retries = 0;
    int32_t* result = nullptr;
    uint64_t* result_cost = nullptr;  // scored runs: cost of each sorted row
    const bool score = opt.score && !hash_mode && opt.sort;
    if (score && opt.cap > kTopkMax)
        return fail(DM_ERR_UNSUPPORTED, "scored enumeration keeps at most " + std::to_string(kTopkMax) + " rows");
    // frees the run's own result buffers on every early return
    struct ResultGuard {
        const dm_context* ctx;
        int32_t** r;
        uint64_t** c;
        hipStream_t s;
        ~ResultGuard() {
            dev_free(ctx, *r, s);
            dev_free(ctx, *c, s);
        }
    } result_guard{ctx, &result, &result_cost, s};

    // Step 0 straight from the motif table, with no join launch: the identity
    // table joined with a motif keyed at position 0 whose new columns are
    // positions 1..L-1 in order, with nothing to check, is the motif table's
    // slice of the root range (its rows are injective and grouped by the key
    // in ascending order), so the next step reads the table in place.  Over
    // every root the slice is the whole table; over a range its first row
    // and length come from the table's index on the device.
    bool zc0 = false;
    const int32_t* zc_base = nullptr;
    const int32_t* zc_offs = nullptr;
    int64_t zc_stride = 0, zc_rows = 0;
    const bool full_range = v0 == 0 && v1 == dg->n;
    {
        const StepDesc& d0 = steps[0];
        if (d0.motif >= 0 && !score && !opt.induced && (full_range || nsteps > 1) && d0.key_pos == 0 &&
            d0.n_eq == 0 && d0.n_edge == 0 && !(nsteps == 1 && hash_mode)) {
            const MotifTable& t = dg->tab[d0.motif][0];
            bool ident = d0.n_new == t.size - 1 && t.rows > 0 && t.cols[0] != nullptr;
            for (int q = 0; q < d0.n_new && ident; q++) ident = d0.new_pos[q] == q + 1;
            for (int q = 1; q < t.size && ident; q++) ident = t.cols[q] == t.cols[0] + (size_t)q * (size_t)t.stride;
            if (ident) {
                zc0 = true;
                zc_base = t.cols[0];
                zc_offs = t.offs;
                zc_stride = t.stride;
                zc_rows = t.rows;
            }
        }
    }

    // profiling: events 0/1 around the join launches (one span: a marker
    // between dependent launches would cost more than the boundary it
    // measures), 2/3 around the LDS sort tiers, 4/5 around the merge tier
    const int first_launch = zc0 ? 1 : 0;
    if (opt.profile) {
        while (ws.prof.size() < (size_t)6) {
            hipEvent_t e;
            DM_HIP(hipEventCreate(&e));
            ws.prof.push_back(e);
        }
    }

    for (;;) {
        for (int b = 0; b < 2; b++) DM_TRY(ws.ensure_buf(b, cap[b] * k));
        // use the whole buffer unless the caller pinned the first-attempt capacity
        if (opt.initial_rows <= 0 || retries > 0)
            for (int b = 0; b < 2; b++) cap[b] = ws.buf_elems[b] / k;
        if (score)
            for (int b = 0; b < 2; b++) DM_TRY(ws.ensure_cbuf(b, cap[b]));
        int64_t maxcap = std::max<int64_t>(std::max(cap[0], cap[1]), (int64_t)dg->n);
        DM_TRY(ws.ensure_status(maxcap / 64 + 2));
        // the control block starts clear; a step 0 read in place over every
        // root has its row count set in the same launch
        if (zc0 && full_range)
            DM_HIP(launch_clear_set_u64((uint64_t*)ws.ctrl_d, sizeof(Control) / 8,
                                        (int64_t)(offsetof(Control, counts) / 8 + 1), (uint64_t)zc_rows, s));
        else
            DM_HIP(launch_fill_u64((uint64_t*)ws.ctrl_d, 0, sizeof(Control) / 8, s));
        if (ws.ev[0]) DM_HIP(hipEventRecord(ws.ev[0], s));
        bool redo = false;
        for (int i = 0; i < nsteps; i++) {
            const int ib = (i - 1) & 1, ob = i & 1;
            if (i == 0 && zc0) {
                if (!full_range) DM_HIP(launch_slice_rows(zc_offs, v0, v1, &ws.ctrl_d->counts[1], &ws.ctrl_d->slice_row0, s));
                if (opt.profile && nsteps == 1) {
                    DM_HIP(hipEventRecord(ws.prof[0], s));
                    DM_HIP(hipEventRecord(ws.prof[1], s));
                }
                continue;
            }
            EjfArgs a;
            std::memset(&a, 0, sizeof a);
            a.st = steps[i];
            if (a.st.motif >= 0) a.tbl = dg->table_dev_step(a.st);
            a.g = dg->graph_dev();
            const bool from_table = i == 1 && zc0;  // the input is the motif table of step 0
            a.in = i == 0 ? nullptr : (from_table ? zc_base : ws.buf[ib]);
            a.in_stride = i == 0 ? 0 : (from_table ? zc_stride : cap[ib]);
            a.in_cap = i == 0 ? 0 : (from_table ? zc_rows : cap[ib]);
            a.in_row0 = (from_table && !full_range) ? &ws.ctrl_d->slice_row0 : nullptr;
            a.n_in = &ws.ctrl_d->counts[i];
            a.id_begin = v0;
            a.id_count = v1 - v0;
            a.out = ws.buf[ob];
            a.out_stride = cap[ob];
            a.out_cap = cap[ob];
            a.n_out = &ws.ctrl_d->counts[i + 1];
            a.overflow = &ws.ctrl_d->overflow[i];
            a.status = ws.status;
            DM_TRY(ws.next_epoch(&a.epoch));
            a.ticket = ws.tickets + a.epoch;
            const bool last = i == nsteps - 1;
            a.mode = (last && hash_mode) ? EJF_HASH : EJF_WRITE;
            a.hash_acc = ws.ctrl_d->hash;
            a.induced = opt.induced ? 1 : 0;
            // rows with many candidates of uneven number (large key groups, the
            // runs of a two-key join): the wave tests candidates, not rows
            if (a.st.motif >= 0 && !score)
                a.cand_par = (a.tbl.pair_offs != nullptr || a.tbl.rows >= 8 * (int64_t)dg->n) ? 1 : 0;
            a.w = wait_ctl(ws.ctx, &ws.ctrl_d->abort, &ws.ctrl_d->diag, opt.wait_limit_us);
            a.diag_pattern = -1;
            a.diag_step = i;
            if (score) {
                a.vcost = dg->vcost;
                a.ecost = dg->ecost;
                a.in_cost = i == 0 ? nullptr : ws.cbuf[ib];
                a.out_cost = ws.cbuf[ob];
            }
            for (int c = 0; c < k; c++) a.pv[c] = (uint8_t)std::max(plan.pv_of[c], 0);
            const double est_in = i == 0 ? (double)(v1 - v0) : est[i - 1];
            const int64_t in_cap = i == 0 ? (int64_t)(v1 - v0) : a.in_cap;
            const int blk = ejf_block_for(a.st.c_in, block);
            if (opt.profile && i == first_launch) DM_HIP(hipEventRecord(ws.prof[0], s));
            DM_HIP(launch_ejf(a, blk, ejf_grid(in_cap, est_in, blk), s));
            if (opt.profile && i == nsteps - 1) DM_HIP(hipEventRecord(ws.prof[1], s));
            if (sync_mode && !(last && hash_mode)) {
                DM_HIP(hipMemcpyAsync(ws.ctrl_h, ws.ctrl_d, sizeof(Control), hipMemcpyDeviceToHost, s));
                DM_HIP(hipStreamSynchronize(s));
                DM_TRY(check_abort(ws.ctrl_h->abort, ws.ctrl_h->diag, "join step"));
                const int64_t need = ws.ctrl_h->counts[i + 1];
                if (need > cap[ob]) {
                    // grow the output buffer only (the input stays intact) and redo
                    if (ws.fixed)
                        return fail(DM_ERR_BUDGET_EXCEEDED, "intermediate table of " + std::to_string(need) +
                                                                " rows does not fit the fixed scratch");
                    if (need > budget_rows)
                        return fail(DM_ERR_BUDGET_EXCEEDED, "intermediate table of " + std::to_string(need) +
                                                                " rows exceeds the memory budget");
                    int64_t nc = need + need / 8 + 1024;
                    dev_free(ctx, ws.buf[ob], s);
                    ws.buf[ob] = nullptr;
                    ws.buf_elems[ob] = 0;
                    DM_TRY(ws.ensure_buf(ob, nc * k));
                    cap[ob] = ws.buf_elems[ob] / k;
                    if (score) DM_TRY(ws.ensure_cbuf(ob, cap[ob]));
                    DM_TRY(ws.ensure_status(cap[ob] / 64 + 2));
                    DM_HIP(launch_fill_i32(&ws.ctrl_d->overflow[i], 0, 1, s));
                    retries++;
                    i--;  // rerun this step
                    continue;
                }
            }
        }
        const int lb = (nsteps - 1) & 1;
        // one readback of the join counts: the result is allocated at its exact
        // size (a buffer sized by the table's capacity would hold as much as
        // the largest table this workspace ever grew to)
        if (!(!hash_mode && opt.sort) && ws.ev[1]) DM_HIP(hipEventRecord(ws.ev[1], s));
        DM_HIP(hipMemcpyAsync(ws.ctrl_h, ws.ctrl_d, sizeof(Control), hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        const Control& c = *ws.ctrl_h;
        DM_TRY(check_abort(c.abort, c.diag, "join step"));
        int first_over = -1;
        for (int i = 0; i < nsteps; i++)
            if (c.overflow[i]) {
                first_over = i;
                break;
            }
        if (first_over >= 0) {
            if (sync_mode) return fail(DM_ERR_INTERNAL, "overflow in exact-sizing mode");
            // counts are exact up to the first overflowing step: size from them and rerun step by step
            int64_t need = 0;
            for (int i = 0; i <= first_over; i++) need = std::max<int64_t>(need, c.counts[i + 1]);
            if (ws.fixed)
                return fail(DM_ERR_BUDGET_EXCEEDED, "intermediate table of " + std::to_string(need) +
                                                        " rows does not fit the fixed scratch");
            if (need > budget_rows)
                return fail(DM_ERR_BUDGET_EXCEEDED,
                            "intermediate table of " + std::to_string(need) + " rows exceeds the memory budget");
            int64_t nc = need + need / 8 + 1024;
            cap[0] = std::max(cap[0], nc);
            cap[1] = std::max(cap[1], nc);
            sync_mode = true;
            retries++;
            continue;
        }
        // the final table: the last step's output, or the motif table itself
        // when the plan's only step was taken in place
        const bool fin_table = zc0 && nsteps == 1;
        int32_t* fin = fin_table ? const_cast<int32_t*>(zc_base) : ws.buf[lb];
        const int64_t fin_stride = fin_table ? zc_stride : cap[lb];
        const int64_t fin_cap = fin_table ? zc_rows : cap[lb];
        const int64_t n_final = std::min<int64_t>(c.counts[nsteps], fin_cap);
        bool sort_merged = false;  // the merge tier ran (its launches are timed apart from the LDS tiers)
        bool sort_streamed = false;  // the streaming pass ran
        if (!hash_mode && opt.sort) {
            // canonicalize into a row-major table of exactly the kept rows
            // (a scored run sorts every row: its cap selects by cost afterwards)
            int64_t out_rows = (opt.cap >= 0 && !score) ? std::min<int64_t>(opt.cap, n_final) : n_final;
            dev_free(ctx, result, s);
            result = nullptr;
            if (opt.out_buf) {
                // the caller's buffer: the sort writes the prefix that fits
                out_rows = std::min<int64_t>(out_rows, opt.out_buf_rows);
            } else {
                DM_TRY(dev_alloc(ctx, (void**)&result, sizeof(int32_t) * (size_t)std::max<int64_t>(out_rows * k, 1),
                                 s));
            }
            if (score) {
                dev_free(ctx, result_cost, s);
                result_cost = nullptr;
                DM_TRY(dev_alloc(ctx, (void**)&result_cost, sizeof(uint64_t) * (size_t)std::max<int64_t>(out_rows, 1), s));
            }
            DM_TRY(ws.ensure_sort_scratch(2 * n_final + 2));
            SortJob& job = *ws.job_h;
            std::memset(&job, 0, sizeof job);
            job.in = fin;
            job.in_stride = fin_stride;
            job.in_cap = fin_cap;
            job.n_in = &ws.ctrl_d->counts[nsteps];
            job.out = opt.out_buf ? opt.out_buf : result;
            job.out_rows = out_rows;
            job.scratch_idx = ws.sort_scratch;
            if (score) {
                job.in_cost = ws.cbuf[lb];
                job.out_cost = result_cost;
            }
            job.k = k;
            sort_pack_layout(k, dg->n, &job);
            for (int j = 0; j < k; j++) job.perm[j] = (uint8_t)plan.col_of[j];
            // the job goes with the sort launches (no upload); the merge tier, when
            // needed, reads it from the device
            if (opt.profile) DM_HIP(hipEventRecord(ws.prof[2], s));
            // the streaming pass, unless the last sort of this plan found its
            // segments out of order (then the per-segment tiers take them directly)
            const bool stream = plan.sort_stream != 0;
            // the merge tier's need is read back with the counters below
            bool merge_pending = false;
            DM_TRY(enqueue_sort(ctx, ws, nullptr, 1, v1 - v0, v0, n_final, job.wp, ws.ctrl_d->sort_counters,
                                &ws.ctrl_d->abort, &ws.ctrl_h->sort_counters[1],
                                opt.profile ? &ws.prof[3] : nullptr, &sort_merged, stream ? k : 0, &merge_pending,
                                &job));
            sort_streamed = stream;
            if (ws.ev[1]) DM_HIP(hipEventRecord(ws.ev[1], s));
            // the sort counters, the abort word and its diagnosis: adjacent in Control, one copy
            static_assert(offsetof(Control, abort) == offsetof(Control, sort_counters) + sizeof(Control::sort_counters),
                          "Control: abort must follow sort_counters");
            static_assert(offsetof(Control, diag) == offsetof(Control, abort) + 2 * sizeof(uint32_t),
                          "Control: diag must follow abort");
            const size_t tail = offsetof(Control, diag) + sizeof(WaitDiag) - offsetof(Control, sort_counters);
            DM_HIP(hipMemcpyAsync(ws.ctrl_h->sort_counters, ws.ctrl_d->sort_counters, tail, hipMemcpyDeviceToHost, s));
            DM_HIP(hipStreamSynchronize(s));
            DM_TRY(check_abort(c.abort, c.diag, "sort"));
            if (merge_pending && c.sort_counters[1] > 0) {
                // segments beyond the largest LDS tile: the merge tier, then the counters again
                DM_HIP(hipMemcpyAsync(ws.job_d, ws.job_h, sizeof(SortJob), hipMemcpyHostToDevice, s));
                DM_TRY(enqueue_sort_merge(ctx, ws, ws.job_d, 1, v1 - v0, v0, n_final, job.wp,
                                          ws.ctrl_d->sort_counters, &ws.ctrl_d->abort,
                                          opt.profile ? &ws.prof[4] : nullptr));
                sort_merged = true;
                if (ws.ev[1]) DM_HIP(hipEventRecord(ws.ev[1], s));
                DM_HIP(hipMemcpyAsync(ws.ctrl_h->sort_counters, ws.ctrl_d->sort_counters, tail,
                                      hipMemcpyDeviceToHost, s));
                DM_HIP(hipStreamSynchronize(s));
                DM_TRY(check_abort(c.abort, c.diag, "sort"));
            }
        }
        if (c.sort_counters[3] != 0) return fail(DM_ERR_INTERNAL, "duplicate rows reached the canonical table");
        if (sort_streamed && !plan.cache_key.empty()) {
            // keep the streaming pass while at most 1/16 of the segments need the tiers after it
            const int32_t hint = 16 * (int64_t)c.sort_counters[4] <= (int64_t)(v1 - v0) ? 1 : 0;
            if (hint != plan.sort_stream) ctx->plans.set_sort_stream(plan.cache_key, hint);
        }
        float ms = 0;
        if (ws.ev[0] && ws.ev[1]) (void)hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]);
        o.stats.device_ms = ms;
        o.stats.n_steps = (int32_t)plan.steps.size();
        o.stats.retries = retries;
        o.stats.chunks = 1;
        int64_t bytes = 0;
        int64_t prev_rows = v1 - v0;
        int prev_cols = 1;
        for (int i = 0; i < nsteps; i++) {
            int64_t r = (hash_mode && i == nsteps - 1) ? (int64_t)c.hash[0] : c.counts[i + 1];
            if (i < DM_MAX_PATTERN_VERTICES) o.stats.step_rows[i] = r;
            const int cols = steps[i].c_in + steps[i].n_new;
            // a step taken in place from the motif table moves nothing
            if (!(i == 0 && zc0))
                bytes += 4 * (prev_cols * prev_rows) + ((hash_mode && i == nsteps - 1) ? 0 : 4 * (int64_t)cols * r);
            prev_rows = r;
            prev_cols = cols;
        }
        o.rows = hash_mode ? (int64_t)c.hash[0] : c.counts[nsteps];
        o.stats.join_bytes = bytes;
        if (!hash_mode && opt.sort) {
            o.stats.sort_bytes = 8 * (int64_t)k * o.rows;
            bytes += o.stats.sort_bytes;
        }
        o.stats.bytes_moved = bytes;
        if (opt.profile) {
            float jm = 0;
            (void)hipEventElapsedTime(&jm, ws.prof[0], ws.prof[1]);
            o.stats.join_ms = jm;
            o.stats.join_launches = nsteps - first_launch;
            if (!hash_mode && opt.sort) {
                // the LDS tiers, plus the merge tier when it ran (not the host
                // round trip that decided it)
                float t = 0, tm = 0;
                (void)hipEventElapsedTime(&t, ws.prof[2], ws.prof[3]);
                if (sort_merged) (void)hipEventElapsedTime(&tm, ws.prof[4], ws.prof[5]);
                o.stats.sort_ms = t + tm;
                o.stats.sort_launches = (sort_merged ? 3 : 2) + (sort_streamed ? 1 : 0);  // + the streaming pass
            }
        }
        if (hash_mode) {
            o.hsum = c.hash[1];
            o.hxor = c.hash[2];
        } else if (score && opt.cap >= 0) {
            // the cap best rows by (cost, row): radix selection over the sorted table
            const int64_t kk = std::min<int64_t>(opt.cap, o.rows);
            if (kk > 0) {
                int32_t* top = nullptr;
                uint64_t *top_cost = nullptr, *sel = nullptr;
                DM_TRY(dev_alloc(ctx, (void**)&top, sizeof(int32_t) * (size_t)(kk * k), s));
                std::unique_ptr<int32_t, std::function<void(int32_t*)>> top_guard(
                    top, [ctx, s](int32_t* p) { dev_free(ctx, p, s); });
                DM_TRY(dev_alloc(ctx, (void**)&top_cost, sizeof(uint64_t) * (size_t)kk, s));
                std::unique_ptr<uint64_t, std::function<void(uint64_t*)>> cost_guard(
                    top_cost, [ctx, s](uint64_t* p) { dev_free(ctx, p, s); });
                // scratch: control block, then k costs and k positions
                const size_t scratch = sizeof(TopkCtl) + (sizeof(uint64_t) + sizeof(uint32_t)) * (size_t)kk + 64;
                DM_TRY(dev_alloc(ctx, (void**)&sel, scratch, s));
                std::unique_ptr<uint64_t, std::function<void(uint64_t*)>> sel_guard(
                    sel, [ctx, s](uint64_t* p) { dev_free(ctx, p, s); });
                TopkCtl* ctl = (TopkCtl*)sel;
                uint64_t* sel_cost = (uint64_t*)((char*)sel + ((sizeof(TopkCtl) + 15) & ~(size_t)15));
                uint32_t* sel_pos = (uint32_t*)(sel_cost + kk);
                DM_HIP(launch_topk(result_cost, o.rows, kk, ctl, sel_cost, sel_pos, result, k, top, top_cost, s));
                DM_HIP(hipStreamSynchronize(s));
                o.sorted = top_guard.release();
                o.costs = cost_guard.release();
            }
            o.sorted_rows = kk;
        } else if (opt.sort && opt.out_buf) {
            o.sorted_rows = opt.cap >= 0 ? std::min<int64_t>(opt.cap, o.rows) : o.rows;
            if (o.sorted_rows > opt.out_buf_rows) {
                *out = o;  // the count, for the caller to size its buffer
                return fail(DM_ERR_BUDGET_EXCEEDED, std::to_string(o.sorted_rows) +
                                                        " rows do not fit the caller's buffer of " +
                                                        std::to_string(opt.out_buf_rows));
            }
        } else if (opt.sort) {
            o.sorted = result;
            o.sorted_rows = opt.cap >= 0 ? std::min<int64_t>(opt.cap, o.rows) : o.rows;
            result = nullptr;
            o.costs = result_cost;
            result_cost = nullptr;
        } else {
            o.table = fin;
            o.stride = fin_stride;
        }
        (void)redo;
        *out = o;
        return DM_OK;
    }
}

// Partition schedule over root ranges.  Tables stay grouped by the root image
// in ascending order, so running the plan on consecutive root ranges and
// concatenating the sorted outputs gives the full sorted table.  Ranges are
// split when an intermediate table would exceed the memory budget, and a cap
// is served from the lowest ranges first (early exit).
dm_status run_plan_chunked(dm_context* ctx, Workspace& ws, const dm_datagraph* dg, const Plan& plan,
                           const RunOptions& opt, RunOutput* out) {
    const bool hash_mode = opt.mode == DM_OUT_COUNT_HASH;
    if (!opt.sort && !hash_mode) return run_plan(ctx, ws, dg, plan, opt, out);
    // a scored cap ranks every row by cost: no early exit and no splitting
    if (opt.score && !hash_mode) return run_plan(ctx, ws, dg, plan, opt, out);
    // the caller's root range (default: every data vertex)
    const int32_t r0 = opt.root_end > opt.root_begin ? std::max(opt.root_begin, 0) : 0;
    const int32_t r1 = opt.root_end > opt.root_begin ? std::min(opt.root_end, dg->n) : dg->n;
    const int32_t n = std::max(r1 - r0, 0);
    std::vector<std::pair<int32_t, int32_t>> todo;  // stack, top = lowest range
    // a cap far below the predicted total: start with small root ranges
    int32_t first_chunk = std::max(n, 1);
    if (opt.cap >= 0 && !hash_mode && plan.est_final_rows > 0 && n > 0) {
        const double per_root = plan.est_final_rows / std::max(dg->n, 1);
        const double want = 4.0 * std::max<double>((double)opt.cap, 1.0) + 1024.0;
        if (per_root * n > 4.0 * want) first_chunk = (int32_t)std::max(1.0, std::min((double)n, want / per_root));
    }
    for (int64_t b = r1; b > r0; b -= first_chunk) {
        const int32_t lo = (int32_t)std::max<int64_t>(r0, b - first_chunk);
        todo.emplace_back(lo, (int32_t)b);
    }
    if (todo.empty()) {  // empty root range: an empty table
        RunOutput o;
        *out = o;
        return DM_OK;
    }
    hipStream_t s = ws.stream;
    std::vector<RunOutput> parts;
    auto free_parts = [&]() {
        for (auto& p : parts) dev_free(ctx, p.sorted, s);
        parts.clear();
    };
    int64_t got = 0;
    bool early = false;
    int splits = 0;
    // Result size: the caller's limit, checked as the parts come in.  Without
    // one, the parts and then the one buffer they are joined into take the
    // result's bytes twice; the workspace tables are allocated by then, so from
    // the second part on the kept rows may take 45 % of the free device memory
    // plus what the parts already hold (a tenth kept for the parts' sorts).
    // Either way an oversized result fails early, not at the final allocation.
    const int64_t row_bytes = 4 * (int64_t)std::max(plan.k, 1);
    int64_t max_result_rows = opt.result_limit > 0 ? std::max<int64_t>(opt.result_limit / row_bytes, 1) : -1;
    while (!todo.empty()) {
        auto rg = todo.back();
        todo.pop_back();
        RunOptions o2 = opt;
        o2.root_begin = rg.first;
        o2.root_end = rg.second;
        if (opt.cap >= 0) o2.cap = std::max<int64_t>(opt.cap - got, 0);
        RunOutput part;
        dm_status st = run_plan(ctx, ws, dg, plan, o2, &part);
        if (st == DM_ERR_BUDGET_EXCEEDED && rg.second - rg.first > 1) {
            // split into four sub-ranges, lowest on top of the stack
            const int32_t len = rg.second - rg.first;
            const int32_t q = std::max(1, (len + 3) / 4);
            std::vector<std::pair<int32_t, int32_t>> sub;
            for (int32_t a = rg.first; a < rg.second; a += q) sub.emplace_back(a, std::min(rg.second, a + q));
            for (auto it = sub.rbegin(); it != sub.rend(); ++it) todo.push_back(*it);
            splits++;
            continue;
        }
        if (st != DM_OK) {
            free_parts();
            return st;
        }
        parts.push_back(part);
        got += hash_mode ? part.rows : part.sorted_rows;
        if (!hash_mode) {
            if (max_result_rows < 0 && parts.size() >= 2) {
                size_t fr = 0, tot = 0;
                int64_t held = 0;
                for (auto& q : parts) held += q.sorted_rows * row_bytes;
                if (hipMemGetInfo(&fr, &tot) == hipSuccess)
                    max_result_rows = std::max<int64_t>((int64_t)(0.45 * (double)((int64_t)fr + held)) / row_bytes, 1);
            }
            const int64_t kept = opt.cap >= 0 ? std::min<int64_t>(got, opt.cap) : got;
            if (max_result_rows >= 0 && kept > max_result_rows) {
                free_parts();
                return fail(DM_ERR_BUDGET_EXCEEDED, "result of more than " + std::to_string(max_result_rows) +
                                                        " rows exceeds the memory it may take");
            }
        }
        if (opt.cap >= 0 && !hash_mode && got >= opt.cap && !todo.empty()) {
            early = true;
            break;
        }
    }
    if (parts.size() == 1 && !early) {
        *out = parts[0];
        out->stats.chunks = 1;
        out->stats.retries += splits;
        return DM_OK;
    }
    RunOutput o;
    o.stats = parts.empty() ? RunOutput().stats : parts[0].stats;
    o.stats.chunks = (int32_t)parts.size();
    o.stats.retries = splits;
    int64_t total = 0, rows = 0;
    double dev_ms = 0, join_ms = 0, sort_ms = 0;
    int64_t jb = 0, sb = 0;
    for (auto& p : parts) {
        total += p.rows;
        rows += p.sorted_rows;
        o.hsum += p.hsum;
        o.hxor ^= p.hxor;
        dev_ms += p.stats.device_ms;
        join_ms += p.stats.join_ms;
        sort_ms += p.stats.sort_ms;
        jb += p.stats.join_bytes;
        sb += p.stats.sort_bytes;
    }
    o.stats.device_ms = dev_ms;
    o.stats.join_ms = join_ms;
    o.stats.sort_ms = sort_ms;
    o.stats.join_bytes = jb;
    o.stats.sort_bytes = sb;
    o.stats.bytes_moved = jb + sb;
    o.rows = early ? -1 : total;
    if (!hash_mode) {
        const int64_t keep = opt.cap >= 0 ? std::min<int64_t>(opt.cap, rows) : rows;
        int32_t* dst = nullptr;
        dm_status st = dev_alloc(ctx, (void**)&dst, sizeof(int32_t) * (size_t)std::max<int64_t>(keep * plan.k, 1), s);
        if (st != DM_OK) {
            free_parts();
            return st;
        }
        int64_t at = 0;
        for (auto& p : parts) {
            const int64_t r = std::min<int64_t>(p.sorted_rows, keep - at);
            if (r > 0) {
                hipError_t e = hipMemcpyAsync(dst + at * plan.k, p.sorted, sizeof(int32_t) * (size_t)(r * plan.k),
                                              hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) {
                    dev_free(ctx, dst, s);
                    free_parts();
                    return hip_fail(e, "hipMemcpyAsync");
                }
            }
            at += std::max<int64_t>(r, 0);
        }
        free_parts();
        DM_HIP(hipStreamSynchronize(s));
        o.sorted = dst;
        o.sorted_rows = keep;
    }
    *out = o;
    return DM_OK;
}

}  // namespace dm

using namespace dm;

dm::TableDev dm_datagraph::table_dev(int motif, int key_pos) const {
    TableDev t;
    std::memset(&t, 0, sizeof t);
    const MotifTable& m = tab[motif][key_pos];
    t.base = m.cols[0];
    t.stride = m.stride;
    t.offs = m.offs;
    t.rows = m.rows;
    t.rstride = 1;
    t.size = m.size;
    t.sorted_by = 0;
    t.sorted_max = 0;
    t.pair_offs = t.pair_far = t.pair_start = nullptr;
    return t;
}

dm::TableDev dm_datagraph::table_dev_step(const dm::StepDesc& st) const {
    TableDev t = table_dev(st.motif, st.key_pos);
    const MotifTable& m = tab[st.motif][st.key_pos];
    if (st.n_eq > 0 && m.sec_base && m.sorted_by == st.eq_pos[0] + 1) {
        t.base = m.sec_base;
        if (m.sec_rowmajor) {
            t.stride = 1;
            t.rstride = m.size;
        }
        t.sorted_by = m.sorted_by;
        t.sorted_max = m.sorted_max;
        t.pair_offs = m.run_offs;
        t.pair_far = m.run_far;
        t.pair_start = m.run_start;
    }
    return t;
}

// ------------------------------------------------------------- C ABI

#define DMOTIF_VERSION_STR "dmotif 0.1 (gfx950)"

extern "C" {

const char* dm_version(void) { return DMOTIF_VERSION_STR; }

const char* dm_last_error(void) { return g_err.c_str(); }

dm_status dm_context_create(int32_t device, void* hip_stream, const dm_allocator* alloc, dm_context** out) {
    if (!out) return fail(DM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(DM_ERR_INVALID_ARG, "allocator with a NULL alloc or free callback");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return fail(DM_ERR_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev) return fail(DM_ERR_INVALID_ARG, "device index out of range");
    DM_HIP(hipSetDevice(device));
    auto* c = new dm_context();
    c->device = device;
    if (alloc) {
        c->has_alloc = true;
        c->alloc = *alloc;
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(DM_ERR_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    auto undo = [&](dm_status st) {
        c->ws.release();
        if (c->cancel) (void)hipHostFree(c->cancel);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return st;
    };
    // the cancel word: host memory the device reads coherently while kernels run
    if (hipHostMalloc((void**)&c->cancel, 64, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        c->cancel = nullptr;
        return undo(fail(DM_ERR_DEVICE, "hipHostMalloc of the cancel word failed"));
    }
    __atomic_store_n(c->cancel, 0u, __ATOMIC_SEQ_CST);
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    if (!c->has_alloc) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    }
    (void)hipGetLastError();
    dm_status st = c->ws.init(c, c->stream);
    if (st != DM_OK) return undo(st);
    c->sort_lds_max = sort_max_lds_bytes();
    *out = c;
    return DM_OK;
}

void dm_context_destroy(dm_context* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    ctx->ws.release();
    flush_blocks(ctx);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->blocks.ev) (void)hipEventDestroy(ctx->blocks.ev);
    if (ctx->cancel) (void)hipHostFree(ctx->cancel);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

dm_status dm_context_cancel(dm_context* ctx, int32_t flag) {
    if (!ctx || !ctx->cancel) return fail(DM_ERR_INVALID_ARG, "NULL context");
    __atomic_store_n(ctx->cancel, flag ? 1u : 0u, __ATOMIC_SEQ_CST);
    return DM_OK;
}

}  // extern "C"

// ------------------------------------------------------------- data graph

static void free_tables(dm_datagraph* dg) {
    hipStream_t s = dg->ctx->stream;
    const dm_context* ctx = dg->ctx;
    for (int m = 0; m < kNumMotifs; m++)
        for (int j = 0; j < 6; j++) {
            MotifTable& t = dg->tab[m][j];
            for (int q = 0; q < 4; q++) dev_free(ctx, t.owned[q], s);
            t = MotifTable();
        }
}

// Drop one motif's tables from the database.
static void free_motif(dm_datagraph* dg, int m) {
    hipStream_t s = dg->ctx->stream;
    const dm_context* ctx = dg->ctx;
    for (int j = 0; j < 6; j++) {
        MotifTable& t = dg->tab[m][j];
        for (int q = 0; q < 4; q++) dev_free(ctx, t.owned[q], s);
        t = MotifTable();
    }
    dg->motif_bits &= ~(1u << m);
    dg->mask_built &= ~motif_info(m).bit;
    dg->stats.rows[m] = 0;
}

static void free_datagraph(dm_datagraph* dg) {
    if (!dg) return;
    hipStream_t s = dg->ctx->stream;
    const dm_context* ctx = dg->ctx;
    free_tables(dg);
    dev_free(ctx, dg->vcost, s);
    dev_free(ctx, dg->ecost, s);
    dev_free(ctx, dg->row_ptr, s);
    dev_free(ctx, dg->src, s);  // src and col share one allocation (src first)
    dev_free(ctx, dg->bitmap, s);
    // the frees are ordered on the context stream after the work queued there
    delete dg;
}

static NormPattern motif_pattern(int m) {
    const MotifInfo& mi = motif_info(m);
    NormPattern p;
    p.k = mi.size;
    if (mi.general) {
        for (int e = 0; e < mi.n_edges; e++)
            p.edges.emplace_back(std::min(mi.edges[e][0], mi.edges[e][1]), std::max(mi.edges[e][0], mi.edges[e][1]));
    } else {
        for (int i = 0; i + 1 < mi.size; i++) p.edges.emplace_back(i, i + 1);
        if (mi.cycle) p.edges.emplace_back(0, mi.size - 1);
    }
    std::sort(p.edges.begin(), p.edges.end());
    return p;
}

// Does the graph (CSR with ascending, merged lists) contain a 4-cycle?  Two
// distinct 2-paths v-u-w and v-u'-w close one.  1 / 0, or -1 when the check
// would walk more than 2e7 2-paths (the caller decides on the device).
static int host_has_4cycle(const std::vector<int32_t>& rp, const std::vector<int32_t>& col, int32_t n) {
    double work = 0;
    for (int32_t v = 0; v < n; v++) {
        const double d = rp[v + 1] - rp[v];
        work += d * d;
    }
    if (work > 2e7) return -1;
    std::vector<int32_t> seen((size_t)n, -1);
    for (int32_t v = 0; v < n; v++)
        for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
            const int32_t u = col[i];
            for (int32_t j = rp[u]; j < rp[u + 1]; j++) {
                const int32_t w = col[j];
                if (w == v) continue;
                if (seen[w] == v) return 1;
                seen[w] = v;
            }
        }
    return 0;
}

// Res(M4-1), the claw, for both of its key positions (centre, leaf) straight
// from the CSR: the same rows Algorithm 2's joins produce (every embedding of
// the claw), sized on the host from the degree sequence and indexed on the
// device (count, scan, fill), so the build reads nothing back.  Returns
// DM_ERR_UNSUPPORTED when the host has no degree sequence or the table would
// not fit int32 offsets (the join-based build then runs instead).
static dm_status build_claw_direct(dm_datagraph* dg) {
    dm_context* ctx = dg->ctx;
    hipStream_t s = ctx->stream;
    Workspace& ws = ctx->ws;
    const int32_t n = dg->n;
    if ((int32_t)dg->host_row_ptr.size() != n + 1 || n <= 0) return DM_ERR_UNSUPPORTED;
    double rows_d = 0;
    for (int32_t v = 0; v < n; v++) {
        const double d = dg->host_row_ptr[v + 1] - dg->host_row_ptr[v];
        rows_d += d * (d - 1) * (d - 2);
    }
    if (rows_d >= (double)INT32_MAX) return DM_ERR_UNSUPPORTED;
    const int64_t rows = (int64_t)rows_d;
    const int m = MOT_K13;
    int32_t* cnt = nullptr;
    DM_TRY(dev_alloc(ctx, (void**)&cnt, sizeof(int32_t) * (size_t)(n + 1), s));
    struct Tmp {
        const dm_context* ctx;
        int32_t* p;
        hipStream_t s;
        ~Tmp() { dev_free(ctx, p, s); }
    } tmp{ctx, cnt, s};
    const int64_t tiles = (int64_t)(n + 1) / 1024 + 2;
    DM_TRY(ws.ensure_status(tiles));
    for (int j = 0; j < 2; j++) {
        MotifTable& t = dg->tab[m][j];
        t.size = 4;
        t.rows = rows;
        int32_t* data = nullptr;
        int32_t* offs = nullptr;
        DM_TRY(dev_alloc(ctx, (void**)&data, sizeof(int32_t) * (size_t)std::max<int64_t>(rows * 4, 1), s));
        t.owned[0] = data;
        DM_TRY(dev_alloc(ctx, (void**)&offs, sizeof(int32_t) * (size_t)(n + 1), s));
        t.owned[1] = offs;
        t.stride = std::max<int64_t>(rows, 1);
        for (int q = 0; q < 4; q++) t.cols[q] = data + (size_t)q * (size_t)t.stride;
        t.offs = offs;
        DM_HIP(launch_claw_count(dg->row_ptr, dg->col, n, j, cnt, s));
        uint32_t ep = 0;
        DM_TRY(ws.next_epoch(&ep));
        DM_HIP(launch_scan_i32(cnt, offs, n, &ws.ctrl_d->counts[0], ws.status, ws.tickets, ep,
                               wait_ctl(ctx, &ws.ctrl_d->abort, &ws.ctrl_d->diag, 0), s));
        DM_HIP(launch_claw_fill(dg->row_ptr, dg->col, n, j, offs, t.stride, data, s));
    }
    dg->motif_bits |= 1u << m;
    dg->mask_built |= motif_info(m).bit;
    dg->stats.rows[m] = (double)rows;
    return DM_OK;
}

// Build Res(M) for motif m (every key position) by running Algorithm 1 on
// the motif itself with the motifs already in the database (Algorithm 2).
// A path table keyed at one end: a second copy, same offsets, with every key
// group ordered by the other end, so that a join knowing both ends (a
// cycle's closing step) binary-searches the group for its run.  The table
// itself keeps the joins' order (paths extended from it come out in label
// order, which the sort skips).  A key group holds at most d (d-1)^(L-2)
// rows (d = the largest degree): groups up to the LDS tile are sorted one
// workgroup each, else (paths up to 6 vertices) only the groups of at most
// 64 rows, one thread each.
static dm_status build_second_copy(dm_datagraph* dg, MotifTable& t) {
    dm_context* ctx = dg->ctx;
    hipStream_t s = ctx->stream;
    const int L = t.size;
    const double d = std::max(dg->max_degree, 1);
    const double bound = d * std::pow(std::max(d - 1.0, 1.0), L - 2);
    const bool lds = bound <= (double)kGroupSortLds;
    int32_t cap = 1;  // LDS pairs: the group-size bound rounded up to a power of two
    while (lds && cap < (int32_t)bound) cap <<= 1;
    if (!lds && L > 6) return DM_OK;
    int32_t* sec = nullptr;
    const size_t bytes = sizeof(int32_t) * (size_t)t.stride * (size_t)L;
    DM_TRY(dev_alloc(ctx, (void**)&sec, bytes, s));
    t.owned[2] = sec;
    if (lds) {
        // row-major: a run's candidates are a few consecutive rows, one or two
        // cache lines instead of one per column
        DM_HIP(launch_group_sort_lds(t.offs, dg->n, t.stride, L, L - 1, t.cols[0], sec, cap, s));
        t.sec_rowmajor = true;
    } else {
        DM_HIP(hipMemcpyAsync(sec, t.cols[0], bytes, hipMemcpyDeviceToDevice, s));
        DM_HIP(launch_group_sort(t.offs, dg->n, t.stride, L, L - 1, sec, s));
    }
    t.sec_base = sec;
    t.sorted_by = L;
    t.sorted_max = lds ? cap : kGroupSortMax;
    if (lds && t.rows > 0 && t.rows < INT32_MAX) {
        // run index: per key, the distinct far ends and where their runs
        // start (flags, their scan, then the runs and the per-key offsets);
        // sized for one run per row, so no count is read back
        Workspace& ws = ctx->ws;
        const int64_t rows = t.rows;
        const size_t a256 = 256;
        auto al = [&](size_t x) { return (x + a256 - 1) / a256 * a256; };
        const size_t b_rows = al(sizeof(int32_t) * (size_t)rows), b_offs = al(sizeof(int32_t) * (size_t)(dg->n + 1));
        int32_t* blk = nullptr;
        DM_TRY(dev_alloc(ctx, (void**)&blk, 2 * b_rows + b_offs, s));
        t.owned[3] = blk;
        t.run_far = blk;
        t.run_start = (int32_t*)((char*)blk + b_rows);
        t.run_offs = (int32_t*)((char*)blk + 2 * b_rows);
        int32_t* tmp = nullptr;
        DM_TRY(dev_alloc(ctx, (void**)&tmp, 2 * b_rows, s));
        struct Tmp {
            const dm_context* ctx;
            int32_t* p;
            hipStream_t s;
            ~Tmp() { dev_free(ctx, p, s); }
        } tmp_guard{ctx, tmp, s};
        int32_t* flags = tmp;
        int32_t* idx = (int32_t*)((char*)tmp + b_rows);
        const int64_t tiles = rows / 1024 + 2;
        DM_TRY(ws.ensure_status(tiles));
        DM_HIP(launch_run_flags(sec, rows, L, L - 1, flags, s));
        uint32_t ep = 0;
        DM_TRY(ws.next_epoch(&ep));
        DM_HIP(launch_scan_i32(flags, idx, rows, &ws.ctrl_d->counts[0], ws.status, ws.tickets, ep,
                               wait_ctl(ctx, &ws.ctrl_d->abort, &ws.ctrl_d->diag, 0), s));
        DM_HIP(launch_run_fill(sec, rows, L, L - 1, flags, idx, t.run_far, t.run_start, s));
        DM_HIP(launch_run_offs(t.offs, dg->n, rows, idx, &ws.ctrl_d->counts[0], t.run_offs, s));
    }
    return DM_OK;
}

static dm_status build_motif(dm_datagraph* dg, int m) {
    if (m == MOT_K13) {
        const dm_status st = build_claw_direct(dg);
        if (st != DM_ERR_UNSUPPORTED) return st;
        free_motif(dg, m);  // nothing half-built stays behind
    }
    dm_context* ctx = dg->ctx;
    hipStream_t s = ctx->stream;
    const MotifInfo& mi = motif_info(m);
    NormPattern p = motif_pattern(m);
    for (int j = 0; j < motif_key_positions(m); j++) {
        Plan plan;
        std::string err;
        dm_status st = plan_pattern(p, j, dg->motif_bits, &dg->stats, &plan, &err);
        if (st != DM_OK) return fail(st, err);
        RunOptions opt;
        opt.sort = false;
        RunOutput ro;
        DM_TRY(run_plan(ctx, ctx->ws, dg, plan, opt, &ro));
        MotifTable& t = dg->tab[m][j];
        t.size = mi.size;
        t.rows = ro.rows;
        int32_t* data = nullptr;
        int32_t* offs = nullptr;
        DM_TRY(dev_alloc(ctx, (void**)&data, sizeof(int32_t) * (size_t)std::max<int64_t>(ro.rows * mi.size, 1), s));
        DM_TRY(dev_alloc(ctx, (void**)&offs, sizeof(int32_t) * (size_t)(dg->n + 1), s));
        t.owned[0] = data;
        t.owned[1] = offs;
        int32_t colmap[kMaxMotif];
        for (int q = 0; q < mi.size; q++) colmap[q] = plan.col_of[q];
        // the final count lives in the control block (device); reuse it for the gather
        const int64_t* n_dev = &ctx->ws.ctrl_d->counts[plan.steps.size()];
        DM_HIP(launch_gather_cols(ro.table, ro.stride, n_dev, ro.rows, colmap, mi.size, data,
                                  std::max<int64_t>(ro.rows, 1), s));
        t.stride = std::max<int64_t>(ro.rows, 1);
        for (int q = 0; q < mi.size; q++) t.cols[q] = data + (size_t)q * (size_t)t.stride;
        DM_HIP(launch_offsets(t.cols[j], n_dev, ro.rows, dg->n, offs, s));
        t.offs = offs;
        if (!mi.general && !mi.cycle && j == 0 && mi.size >= 3 && ro.rows > 0) DM_TRY(build_second_copy(dg, t));
    }
    dg->motif_bits |= 1u << m;
    dg->mask_built |= mi.bit;
    dg->stats.rows[m] = (double)dg->tab[m][0].rows;
    return DM_OK;
}

// host_csr (optional): receives row_ptr and col, read back with the edge
// count, and *has_c4 whether the graph has a 4-cycle (1 / 0, -1 when a vertex
// of degree above 16 left it undecided).
static dm_status ingest(dm_datagraph* dg, const dm_graph_desc* gd,
                        std::pair<std::vector<int32_t>, std::vector<int32_t>>* host_csr = nullptr,
                        int* has_c4 = nullptr) {
    dm_context* ctx = dg->ctx;
    hipStream_t s = ctx->stream;
    Workspace& ws = ctx->ws;
    const int32_t n = gd->n_vertices;
    const int64_t m = gd->n_edges;
    if ((int64_t)2 * m >= (int64_t)INT32_MAX) return fail(DM_ERR_UNSUPPORTED, "more than 2^30 edges");
    int32_t *d_edges = nullptr, *deg = nullptr, *tmp_ptr = nullptr, *tmp = nullptr, *cursor = nullptr,
            *udeg = nullptr, *big = nullptr, *flags = nullptr;
    // every scratch array in one allocation (sizes are host-known bounds)
    const int64_t emax = std::max<int64_t>(2 * m, 1);
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t vbytes = a256(sizeof(int32_t) * (size_t)(n + 1));
    const size_t ebytes = a256(sizeof(int32_t) * (size_t)emax);
    const size_t scr_bytes = 256 + 2 * ebytes + 5 * vbytes;
    char* scr = nullptr;
    auto cleanup = [&]() { dev_free(ctx, scr, s); };
    dm_status st = DM_OK;
    do {
        // flags: [0] range error bits, [1] big-list count, [2] max degree
        if ((st = dev_alloc(ctx, (void**)&scr, scr_bytes, s))) break;
        {
            char* q = scr;
            // the arrays that start at zero first, so one fill clears them
            flags = (int32_t*)q, q += 256;
            deg = (int32_t*)q, q += vbytes;
            tmp_ptr = (int32_t*)q, q += vbytes;
            cursor = (int32_t*)q, q += vbytes;
            udeg = (int32_t*)q, q += vbytes;
            d_edges = (int32_t*)q, q += ebytes;
            tmp = (int32_t*)q, q += ebytes;
            big = (int32_t*)q;
        }
        // the control block (counts, the abort word of the scans' look-backs) starts clear
        if (launch_fill_u64((uint64_t*)ws.ctrl_d, 0, sizeof(Control) / 8, s) ||
            launch_fill_i32(flags, 0, (int64_t)((256 + 4 * vbytes) / sizeof(int32_t)), s)) {
            st = fail(DM_ERR_DEVICE, "fill launch failed");
            break;
        }
        // the pinned staging buffer carries the edges up and, at the end, the
        // results back: a copy from pageable memory would wait for the host
        const size_t off_rp = 128, off_col = off_rp + a256(sizeof(int32_t) * (size_t)(n + 1));
        const size_t need = off_col + (host_csr ? sizeof(int32_t) * (size_t)emax : 0);
        const size_t edge_bytes = sizeof(int32_t) * 2 * (size_t)m;
        if ((st = ws.ensure_stage(std::max(need, edge_bytes)))) break;
        if (m > 0) {
            std::memcpy(ws.stage_h, gd->edges, edge_bytes);
            if (hipMemcpyAsync(d_edges, ws.stage_h, edge_bytes, hipMemcpyHostToDevice, s)) {
                st = fail(DM_ERR_DEVICE, "edge upload failed");
                break;
            }
        }
        if (launch_ingest_count(d_edges, m, n, deg, flags, s)) {
            st = fail(DM_ERR_DEVICE, "ingest_count launch failed");
            break;
        }
        // exclusive scan of raw degrees -> tmp_ptr
        int64_t tiles = (int64_t)(n + 1) / 1024 + 2;
        if ((st = ws.ensure_status(tiles))) break;
        uint32_t ep = 0;
        if ((st = ws.next_epoch(&ep))) break;
        if (launch_scan_i32(deg, tmp_ptr, n, &ws.ctrl_d->counts[0], ws.status, ws.tickets, ep,
                            wait_ctl(ctx, &ws.ctrl_d->abort, &ws.ctrl_d->diag, 0), s)) {
            st = fail(DM_ERR_DEVICE, "scan launch failed");
            break;
        }
        // Every buffer below is sized by host-known bounds (at most 2m directed
        // edges before and after merging repeats), so the pipeline runs to the
        // end without a readback; range and degree errors are read with the
        // edge count once, at the end (the kernels skip the bad entries).
        if (launch_ingest_scatter(d_edges, m, n, tmp_ptr, cursor, tmp, s) ||
            launch_ingest_sort_small(tmp_ptr, tmp, n, udeg, big, flags + 1, s) ||
            launch_ingest_sort_big(tmp_ptr, tmp, udeg, big, flags + 1, flags, s)) {
            st = fail(DM_ERR_DEVICE, "ingest sort launch failed");
            break;
        }
        if ((st = dev_alloc(ctx, (void**)&dg->row_ptr, sizeof(int32_t) * (size_t)(n + 1), s))) break;
        if ((st = ws.next_epoch(&ep))) break;
        if (launch_scan_i32(udeg, dg->row_ptr, n, &ws.ctrl_d->counts[1], ws.status, ws.tickets, ep,
                            wait_ctl(ctx, &ws.ctrl_d->abort, &ws.ctrl_d->diag, 0), s)) {
            st = fail(DM_ERR_DEVICE, "scan launch failed");
            break;
        }
        // src | col in one block (column stride emax): Res(M2) is then an
        // ordinary 2-column SoA table
        if ((st = dev_alloc(ctx, (void**)&dg->src, sizeof(int32_t) * 2 * (size_t)emax, s))) break;
        dg->col = dg->src + emax;
        if (launch_ingest_compact(tmp_ptr, tmp, dg->row_ptr, n, dg->col, dg->src, flags + 2, s)) {
            st = fail(DM_ERR_DEVICE, "compact launch failed");
            break;
        }
        if (has_c4 && launch_c4_check(dg->row_ptr, dg->col, n, flags + 3, s)) {
            st = fail(DM_ERR_DEVICE, "4-cycle check launch failed");
            break;
        }
        if (n <= 32768 && n > 0) {
            dg->words_per_row = (n + 31) / 32;
            int64_t words = (int64_t)n * dg->words_per_row;
            if ((st = dev_alloc(ctx, (void**)&dg->bitmap, sizeof(uint32_t) * (size_t)words, s))) break;
            (void)launch_fill_i32((int32_t*)dg->bitmap, 0, words, s);
            if (launch_bitmap_set(dg->src, dg->col, &ws.ctrl_d->counts[1], emax, dg->words_per_row, dg->bitmap, s)) {
                st = fail(DM_ERR_DEVICE, "bitmap launch failed");
                break;
            }
        }
        // one readback through the pinned staging buffer (its edges were
        // copied up before any kernel below ran): edge count, flags, row
        // offsets, and the adjacency lists when the caller wants them
        char* H = ws.stage_h;
        HostGather hg;
        std::memset(&hg, 0, sizeof hg);
        auto add = [&](const void* src, size_t off, size_t bytes) {
            hg.src[hg.n] = src;
            hg.dst[hg.n] = H + off;
            hg.bytes[hg.n] = (int64_t)bytes;
            hg.n++;
        };
        add(&ws.ctrl_d->counts[1], 0, sizeof(int64_t));
        add(&ws.ctrl_d->abort, 8, sizeof(uint32_t));
        add(flags, 64, 16 * sizeof(int32_t));
        add(dg->row_ptr, off_rp, sizeof(int32_t) * ((size_t)n + 1));
        if (host_csr) add(dg->col, off_col, sizeof(int32_t) * (size_t)emax);
        const bool copied = launch_gather_to_host(hg, s) == hipSuccess;
        if (!copied || hipStreamSynchronize(s) != hipSuccess) {
            st = fail(DM_ERR_DEVICE, "ingest readback failed");
            break;
        }
        int64_t nnz = 0;
        int32_t hflags[16];
        std::memcpy(&nnz, H, sizeof nnz);
        std::memcpy(hflags, H + 64, sizeof hflags);
        uint32_t habort = 0;
        std::memcpy(&habort, H + 8, sizeof habort);
        if (habort) {
            WaitDiag d;
            std::memset(&d, 0, sizeof d);
            (void)hipMemcpy(&d, &ws.ctrl_d->diag, sizeof d, hipMemcpyDeviceToHost);
            st = check_abort(habort, d, "data-graph ingest");
            break;
        }
        // the degree sequence stays on the host (it sizes tables built from the CSR)
        dg->host_row_ptr.assign((const int32_t*)(H + off_rp), (const int32_t*)(H + off_rp) + (n + 1));
        if (hflags[0] & 1) {
            st = fail(DM_ERR_VERTEX_RANGE, "data graph vertex id out of range");
            break;
        }
        if (hflags[0] & 2) {
            st = fail(DM_ERR_UNSUPPORTED, "a vertex degree exceeds 16384");
            break;
        }
        dg->nnz = nnz;
        if (host_csr) {
            host_csr->first = dg->host_row_ptr;
            host_csr->second.assign((const int32_t*)(H + off_col), (const int32_t*)(H + off_col) + nnz);
        }
        dg->max_degree = hflags[2];
        if (has_c4) *has_c4 = hflags[4] ? -1 : (hflags[3] ? 1 : 0);
    } while (0);
    cleanup();
    if (st == DM_OK) {
        // Res(M2): the directed edge table, keyed on its first column = CSR
        MotifTable& t = dg->tab[MOT_P2][0];
        t.size = 2;
        t.rows = dg->nnz;
        t.cols[0] = dg->src;
        t.cols[1] = dg->col;
        t.stride = dg->col - dg->src;
        t.offs = dg->row_ptr;
        dg->stats.n_vertices = n;
        dg->stats.rows[MOT_P2] = (double)dg->nnz;
        dg->stats.avg_degree = n > 0 ? (double)dg->nnz / n : 0.0;
    }
    return st;
}

// ---- persisted motif database
//
// File image (little-endian): "DMOTIFDB", u32 version, u32 reserved, then
// i32 n, i64 nnz, u32 mask_built, u32 motif_bits, f64 stats rows[kNumMotifs], f64
// avg_degree, i32 row_ptr[n+1], i32 col[nnz], then for every built motif
// other than M2 (which is the CSR) and every key position: i64 rows, i32
// size, i32 column data [size][rows] (motif position order), i32 offs[n+1];
// last a u64 FNV-1a checksum of every byte before it.

namespace {

constexpr char kDbMagic[8] = {'D', 'M', 'O', 'T', 'I', 'F', 'D', 'B'};
constexpr uint32_t kDbVersion = 2;

uint64_t fnv1a(const void* p, size_t n, uint64_t h) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) {
        h ^= b[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

struct DbWriter {
    FILE* f;
    uint64_t h = 0xCBF29CE484222325ull;
    bool ok = true;
    void put(const void* p, size_t n) {
        if (!ok || n == 0) return;
        ok = std::fwrite(p, 1, n, f) == n;
        h = fnv1a(p, n, h);
    }
    template <class T>
    void val(const T& v) { put(&v, sizeof v); }
};

struct DbReader {
    const unsigned char* p;
    size_t n, at = 0;
    bool get(void* dst, size_t len) {
        if (len > n - at) return false;
        std::memcpy(dst, p + at, len);
        at += len;
        return true;
    }
    template <class T>
    bool val(T* v) { return get(v, sizeof *v); }
};

}  // namespace

extern "C" {

dm_status dm_datagraph_build(dm_context* ctx, const dm_graph_desc* gd, uint32_t motif_mask, dm_datagraph** out) {
    if (!ctx || !gd || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (gd->n_vertices < 0 || gd->n_edges < 0 || (gd->n_edges > 0 && !gd->edges))
        return fail(DM_ERR_INVALID_ARG, "invalid data graph descriptor");
    DM_HIP(hipSetDevice(ctx->device));
    auto* dg = new dm_datagraph();
    dg->ctx = ctx;
    dg->n = gd->n_vertices;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, ctx->stream);
    const bool aut = (motif_mask == DM_MOTIF_AUTO);
    std::pair<std::vector<int32_t>, std::vector<int32_t>> csr;  // host copy for the AUTO choice
    const auto tb0 = std::chrono::steady_clock::now();
    int c4_dev = -1;
    dm_status st = ingest(dg, gd, aut ? &csr : nullptr, aut ? &c4_dev : nullptr);
    const auto tb1 = std::chrono::steady_clock::now();
    if (st == DM_OK && dg->n > 0) {
        uint32_t want = motif_mask;
        if (aut) {
            // topology-aware set (Sec. VI-B): the square cell on grid-like graphs,
            // the claw on low-degree graphs without 4-cycles (heavy-hex-like)
            // (decided on the device with the ingest, else walked here)
            int c4 = c4_dev >= 0 ? c4_dev : host_has_4cycle(csr.first, csr.second, dg->n);
            if (c4 < 0) {
                // too many 2-paths to check on the host: the cycle table decides
                st = build_motif(dg, MOT_C4);
                c4 = st == DM_OK && dg->tab[MOT_C4][0].rows > 0 ? 1 : 0;
                if (st == DM_OK && !c4) free_motif(dg, MOT_C4);
            }
            if (c4) {
                // with degrees up to 4 also M7, the 7-path keyed at its ends
                // (12-cycles close as one two-key join of two 7-paths); its
                // table is checked against its size after M4 is built
                want = DM_MOTIF_M3 | DM_MOTIF_M4 | DM_MOTIF_C4 | (dg->max_degree <= 4 ? DM_MOTIF_M7 : 0u);
            } else {
                // the claw table has sum_v d(d-1)(d-2) rows: only for low degrees
                double claws = 0;
                for (int32_t v = 0; v < dg->n; v++) {
                    const double d = csr.first[v + 1] - csr.first[v];
                    claws += d * (d - 1) * (d - 2);
                }
                // with the claw, M7 for the pattern's chains (paths and
                // cycles take a few long slices instead of one join per edge)
                want = claws <= 5e7 ? (DM_MOTIF_M4_1 | (dg->max_degree <= 4 ? DM_MOTIF_M7 : 0u))
                                    : (DM_MOTIF_M3 | DM_MOTIF_M4);
            }
        }
        const int order[] = {MOT_P3, MOT_P4, MOT_P5, MOT_P6, MOT_P7, MOT_C4, MOT_C6, MOT_C12, MOT_K13, MOT_G23, MOT_H18};
        for (int m : order) {
            if (st != DM_OK) break;
            if (!(want & motif_info(m).bit) || ((dg->motif_bits >> m) & 1)) continue;
            if (aut && m == MOT_P7) {
                // M7 only while its table (about M4 x (d-1)^3 rows, x 2 copies) stays moderate
                const double d1 = std::max(dg->max_degree - 1, 1);
                if (dg->stats.rows[MOT_P4] * d1 * d1 * d1 > 5e7) continue;
            }
            st = build_motif(dg, m);
        }
        if (st == DM_OK && aut && !(want & (DM_MOTIF_C4 | DM_MOTIF_M4_1))) {
            // high-degree graph without 4-cycles: the 12-cycle cell when its
            // path table stays moderate (estimated from the growth M3 -> M4)
            double r3 = dg->stats.rows[MOT_P3], r4 = dg->stats.rows[MOT_P4];
            double g = r3 > 0 ? r4 / r3 : 0;
            double est12 = r4 * std::pow(std::max(g, 1.0), 8);
            if (r4 > 0 && est12 < 5e7) st = build_motif(dg, MOT_C12);
        }
    }
    (void)hipEventRecord(e1, ctx->stream);
    const auto tb2 = std::chrono::steady_clock::now();
    if (st == DM_OK) {
        // a scan look-back that gave up leaves its mark in the control block:
        // its abort word and diagnosis come back with the build's last sync
        Control* h = ctx->ws.ctrl_h;
        const size_t at = offsetof(Control, abort), len = offsetof(Control, diag) + sizeof(WaitDiag) - at;
        if (hipMemcpyAsync((char*)h + at, (const char*)ctx->ws.ctrl_d + at, len, hipMemcpyDeviceToHost,
                           ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            st = fail(DM_ERR_DEVICE, "build sync failed");
        else
            st = check_abort(h->abort, h->diag, "data-graph build");
    }
    if (std::getenv("DMOTIF_BUILD_TIMING")) {
        auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        std::fprintf(stderr, "[build] ingest %.3f ms, motif tables (enqueue) %.3f ms, final sync %.3f ms\n",
                     ms(tb0, tb1), ms(tb1, tb2), ms(tb2, std::chrono::steady_clock::now()));
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dg->build_ms = ms;
    if (st != DM_OK) {
        free_datagraph(dg);
        return st;
    }
    *out = dg;
    return DM_OK;
}

dm_status dm_datagraph_free(dm_datagraph* dg) {
    if (!dg) return DM_OK;
    if (dg->servers.load() > 0) return fail(DM_ERR_BUSY, "a server still holds this data graph; stop it first");
    (void)hipSetDevice(dg->ctx->device);
    free_datagraph(dg);
    return DM_OK;
}


dm_status dm_datagraph_save(const dm_datagraph* dg, const char* path) {
    if (!dg || !path) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    DM_HIP(hipSetDevice(dg->ctx->device));
    hipStream_t s = dg->ctx->stream;
    std::vector<int32_t> row_ptr((size_t)dg->n + 1), col((size_t)dg->nnz);
    DM_HIP(hipMemcpyAsync(row_ptr.data(), dg->row_ptr, sizeof(int32_t) * row_ptr.size(), hipMemcpyDeviceToHost, s));
    if (dg->nnz > 0) DM_HIP(hipMemcpyAsync(col.data(), dg->col, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(DM_ERR_INVALID_ARG, std::string("cannot open for writing: ") + path);
    DbWriter w{f};
    w.put(kDbMagic, sizeof kDbMagic);
    w.val(kDbVersion);
    w.val((uint32_t)0);
    w.val(dg->n);
    w.val(dg->nnz);
    w.val(dg->mask_built);
    w.val(dg->motif_bits);
    for (int m = 0; m < kNumMotifs; m++) w.val(dg->stats.rows[m]);
    w.val(dg->stats.avg_degree);
    w.put(row_ptr.data(), sizeof(int32_t) * row_ptr.size());
    w.put(col.data(), sizeof(int32_t) * col.size());
    std::vector<int32_t> buf;
    for (int m = 0; m < kNumMotifs && w.ok; m++) {
        if (m == MOT_P2 || !((dg->motif_bits >> m) & 1)) continue;
        for (int j = 0; j < motif_key_positions(m) && w.ok; j++) {
            const MotifTable& t = dg->tab[m][j];
            w.val(t.rows);
            w.val(t.size);
            buf.resize((size_t)std::max<int64_t>(t.rows, 0));
            for (int q = 0; q < t.size && w.ok; q++) {
                if (t.rows > 0) {
                    DM_HIP(hipMemcpyAsync(buf.data(), t.cols[q], sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s));
                    DM_HIP(hipStreamSynchronize(s));
                }
                w.put(buf.data(), sizeof(int32_t) * buf.size());
            }
            buf.resize((size_t)dg->n + 1);
            DM_HIP(hipMemcpyAsync(buf.data(), t.offs, sizeof(int32_t) * buf.size(), hipMemcpyDeviceToHost, s));
            DM_HIP(hipStreamSynchronize(s));
            w.put(buf.data(), sizeof(int32_t) * buf.size());
        }
    }
    const uint64_t sum = w.h;
    if (w.ok) w.ok = std::fwrite(&sum, 1, sizeof sum, f) == sizeof sum;
    const bool closed = std::fclose(f) == 0;
    if (!w.ok || !closed) return fail(DM_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return DM_OK;
}

dm_status dm_datagraph_load(dm_context* ctx, const char* path, dm_datagraph** out) {
    if (!ctx || !path || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    std::vector<unsigned char> img;
    {
        FILE* f = std::fopen(path, "rb");
        if (!f) return fail(DM_ERR_INVALID_ARG, std::string("cannot open: ") + path);
        unsigned char chunk[1 << 16];
        size_t got;
        while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) img.insert(img.end(), chunk, chunk + got);
        std::fclose(f);
    }
    auto corrupt = [&](const char* why) { return fail(DM_ERR_INVALID_ARG, std::string("not a valid motif database (") + why + "): " + path); };
    if (img.size() < sizeof kDbMagic + 8 + sizeof(uint64_t)) return corrupt("too short");
    uint64_t stored;
    std::memcpy(&stored, img.data() + img.size() - sizeof stored, sizeof stored);
    if (fnv1a(img.data(), img.size() - sizeof stored, 0xCBF29CE484222325ull) != stored) return corrupt("checksum");
    DbReader r{img.data(), img.size() - sizeof stored};
    char magic[8];
    uint32_t version = 0, reserved = 0, mask = 0, bits = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    if (!r.get(magic, 8) || std::memcmp(magic, kDbMagic, 8) != 0) return corrupt("magic");
    if (!r.val(&version) || version != kDbVersion || !r.val(&reserved)) return corrupt("version");
    MotifStats stats;
    if (!r.val(&n) || !r.val(&nnz) || !r.val(&mask) || !r.val(&bits) || n < 0 || nnz < 0 || nnz >= INT32_MAX)
        return corrupt("header");
    for (int m = 0; m < kNumMotifs; m++)
        if (!r.val(&stats.rows[m])) return corrupt("header");
    if (!r.val(&stats.avg_degree)) return corrupt("header");
    std::vector<int32_t> row_ptr((size_t)n + 1), col((size_t)nnz);
    if (!r.get(row_ptr.data(), sizeof(int32_t) * row_ptr.size()) || !r.get(col.data(), sizeof(int32_t) * col.size()))
        return corrupt("graph");
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return corrupt("graph");
    // the edge list of the stored CSR (u < v); ingest rebuilds the device CSR,
    // its source column and the bitmap exactly as a build does
    std::vector<int32_t> edges;
    for (int32_t u = 0; u < n; u++) {
        if (row_ptr[u + 1] < row_ptr[u]) return corrupt("graph");
        for (int32_t i = row_ptr[u]; i < row_ptr[u + 1]; i++) {
            const int32_t v = col[(size_t)i];
            if (v < 0 || v >= n) return corrupt("graph");
            if (u < v) {
                edges.push_back(u);
                edges.push_back(v);
            }
        }
    }
    DM_HIP(hipSetDevice(ctx->device));
    auto* dg = new dm_datagraph();
    dg->ctx = ctx;
    dg->n = n;
    const auto t0 = std::chrono::steady_clock::now();
    dm_graph_desc gd{n, (int64_t)edges.size() / 2, edges.empty() ? nullptr : edges.data()};
    dm_status st = ingest(dg, &gd);
    if (st == DM_OK && dg->nnz != nnz) st = corrupt("graph");
    hipStream_t s = ctx->stream;
    for (int m = 0; m < kNumMotifs && st == DM_OK; m++) {
        if (m == MOT_P2 || !((bits >> m) & 1)) continue;
        for (int j = 0; j < motif_key_positions(m) && st == DM_OK; j++) {
            int64_t rows = 0;
            int32_t size = 0;
            if (!r.val(&rows) || !r.val(&size) || rows < 0 || size != motif_info(m).size) {
                st = corrupt("motif table");
                break;
            }
            MotifTable& t = dg->tab[m][j];
            t.size = size;
            t.rows = rows;
            t.stride = std::max<int64_t>(rows, 1);
            int32_t *data = nullptr, *offs = nullptr;
            if ((st = dev_alloc(ctx, (void**)&data, sizeof(int32_t) * (size_t)(t.stride * size), s))) break;
            t.owned[0] = data;
            if ((st = dev_alloc(ctx, (void**)&offs, sizeof(int32_t) * (size_t)(n + 1), s))) break;
            t.owned[1] = offs;
            std::vector<int32_t> colbuf((size_t)rows);
            for (int q = 0; q < size && st == DM_OK; q++) {
                t.cols[q] = data + (size_t)q * (size_t)t.stride;
                if (!r.get(colbuf.data(), sizeof(int32_t) * colbuf.size())) {
                    st = corrupt("motif table");
                    break;
                }
                for (int32_t v : colbuf)
                    if (v < 0 || v >= n) {
                        st = corrupt("motif table");
                        break;
                    }
                if (st == DM_OK && rows > 0 &&
                    hipMemcpy(t.cols[q], colbuf.data(), sizeof(int32_t) * colbuf.size(), hipMemcpyHostToDevice))
                    st = fail(DM_ERR_DEVICE, "motif table upload failed");
            }
            if (st != DM_OK) break;
            std::vector<int32_t> ob((size_t)n + 1);
            if (!r.get(ob.data(), sizeof(int32_t) * ob.size()) || ob[0] != 0 || ob[n] != rows) {
                st = corrupt("motif index");
                break;
            }
            for (int32_t v = 0; v < n; v++)
                if (ob[v + 1] < ob[v]) {
                    st = corrupt("motif index");
                    break;
                }
            if (st == DM_OK && hipMemcpy(offs, ob.data(), sizeof(int32_t) * ob.size(), hipMemcpyHostToDevice))
                st = fail(DM_ERR_DEVICE, "motif index upload failed");
            t.offs = offs;
            const MotifInfo& mi = motif_info(m);
            if (st == DM_OK && !mi.general && !mi.cycle && j == 0 && size >= 3 && rows > 0)
                st = build_second_copy(dg, t);
        }
    }
    if (st == DM_OK && r.at != r.n) st = corrupt("trailing bytes");
    if (st == DM_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(DM_ERR_DEVICE, "load sync failed");
    if (st != DM_OK) {
        free_datagraph(dg);
        return st;
    }
    dg->motif_bits = bits | 1u;
    dg->mask_built = mask;
    for (int m = 0; m < kNumMotifs; m++)
        if (m != MOT_P2) dg->stats.rows[m] = stats.rows[m];
    dg->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = dg;
    return DM_OK;
}

dm_status dm_datagraph_query(const dm_datagraph* dg, dm_datagraph_info* out) {
    if (!dg || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    std::memset(out, 0, sizeof *out);
    out->n_vertices = dg->n;
    out->n_directed_edges = dg->nnz;
    out->max_degree = dg->max_degree;
    out->has_bitmap = dg->bitmap != nullptr;
    out->motif_mask = dg->mask_built;
    for (int m = 0; m < kNumMotifs; m++) out->motif_rows[m] = (dg->motif_bits >> m) & 1 ? dg->tab[m][0].rows : 0;
    out->build_ms = dg->build_ms;
    return DM_OK;
}

dm_status dm_datagraph_set_costs(dm_datagraph* dg, const uint32_t* vertex_cost, int64_t n_cost_edges,
                                 const int32_t* cost_edges, const uint32_t* edge_cost) {
    if (dg && dg->servers.load() > 0) return fail(DM_ERR_BUSY, "a server holds this data graph");
    if (!dg || n_cost_edges < 0 || (n_cost_edges > 0 && (!cost_edges || !edge_cost)))
        return fail(DM_ERR_INVALID_ARG, "invalid cost arguments");
    DM_HIP(hipSetDevice(dg->ctx->device));
    hipStream_t s = dg->ctx->stream;
    // place each listed edge's cost at both of its CSR positions (host copy of the CSR)
    std::vector<int32_t> row_ptr((size_t)dg->n + 1), col((size_t)dg->nnz);
    DM_HIP(hipMemcpyAsync(row_ptr.data(), dg->row_ptr, sizeof(int32_t) * row_ptr.size(), hipMemcpyDeviceToHost, s));
    if (dg->nnz > 0) DM_HIP(hipMemcpyAsync(col.data(), dg->col, sizeof(int32_t) * col.size(), hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    std::vector<uint32_t> ec((size_t)std::max<int64_t>(dg->nnz, 1), 0u);
    std::vector<char> seen((size_t)std::max<int64_t>(dg->nnz, 1), 0);
    for (int64_t e = 0; e < n_cost_edges; e++) {
        for (int o = 0; o < 2; o++) {
            const int32_t x = cost_edges[2 * e + o], y = cost_edges[2 * e + 1 - o];
            if (x < 0 || y < 0 || x >= dg->n || y >= dg->n)
                return fail(DM_ERR_INVALID_ARG, "cost edge " + std::to_string(e) + " has a vertex out of range");
            auto b = col.begin() + row_ptr[x], en = col.begin() + row_ptr[x + 1];
            auto it = std::lower_bound(b, en, y);
            if (it == en || *it != y)
                return fail(DM_ERR_INVALID_ARG, "cost edge " + std::to_string(e) + " is not an edge of the graph");
            const size_t at = (size_t)(it - col.begin());
            if (seen[at]) return fail(DM_ERR_INVALID_ARG, "cost edge " + std::to_string(e) + " is listed twice");
            seen[at] = 1;
            ec[at] = edge_cost[e];
        }
    }
    DM_TRY(ensure_costs(dg));
    if (vertex_cost)
        DM_HIP(hipMemcpyAsync(dg->vcost, vertex_cost, sizeof(uint32_t) * (size_t)dg->n, hipMemcpyHostToDevice, s));
    else
        DM_HIP(launch_fill_i32((int32_t*)dg->vcost, 0, std::max(dg->n, 1), s));
    DM_HIP(hipMemcpyAsync(dg->ecost, ec.data(), sizeof(uint32_t) * ec.size(), hipMemcpyHostToDevice, s));
    DM_HIP(hipStreamSynchronize(s));
    return DM_OK;
}

dm_status dm_datagraph_copy_csr(const dm_datagraph* dg, int32_t* row_ptr, int32_t* col) {
    if (!dg || !row_ptr || (!col && dg->nnz > 0)) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    DM_HIP(hipSetDevice(dg->ctx->device));
    hipStream_t s = dg->ctx->stream;
    DM_HIP(hipMemcpyAsync(row_ptr, dg->row_ptr, sizeof(int32_t) * (size_t)(dg->n + 1), hipMemcpyDeviceToHost, s));
    if (dg->nnz > 0) DM_HIP(hipMemcpyAsync(col, dg->col, sizeof(int32_t) * (size_t)dg->nnz, hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    return DM_OK;
}

dm_status dm_datagraph_copy_motif(const dm_datagraph* dg, int32_t motif, int32_t key_pos, int32_t* dst,
                                  int64_t max_rows, int64_t* rows, int32_t* width) {
    if (!dg || motif < 0 || motif >= kNumMotifs) return fail(DM_ERR_INVALID_ARG, "bad motif index");
    if (!((dg->motif_bits >> motif) & 1)) return fail(DM_ERR_INVALID_ARG, "motif not built");
    if (key_pos < 0 || key_pos >= motif_key_positions(motif)) return fail(DM_ERR_INVALID_ARG, "bad key position");
    const MotifTable& t = dg->tab[motif][key_pos];
    if (rows) *rows = t.rows;
    if (width) *width = t.size;
    if (!dst) return DM_OK;
    DM_HIP(hipSetDevice(dg->ctx->device));
    hipStream_t s = dg->ctx->stream;
    int64_t r = std::min<int64_t>(max_rows, t.rows);
    if (r <= 0) return DM_OK;
    std::vector<int32_t> colbuf((size_t)r);
    for (int p = 0; p < t.size; p++) {
        DM_HIP(hipMemcpyAsync(colbuf.data(), t.cols[p], sizeof(int32_t) * (size_t)r, hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < r; i++) dst[i * t.size + p] = colbuf[(size_t)i];
    }
    return DM_OK;
}

dm_status dm_plan(const dm_graph_desc* gp, uint32_t motif_mask, int32_t* buf, int32_t buf_cap, int32_t* len) {
    if (!len) return fail(DM_ERR_INVALID_ARG, "len is NULL");
    NormPattern p;
    std::string err;
    dm_status st = normalize_pattern(gp, &p, &err);
    if (st != DM_OK) return fail(st, err);
    Plan plan;
    st = plan_pattern(p, 0, motif_bits_from_mask(motif_mask), nullptr, &plan, &err);
    if (st != DM_OK) return fail(st, err);
    std::vector<int32_t> v = serialize_plan(plan);
    *len = (int32_t)v.size();
    if (!buf || buf_cap < (int32_t)v.size()) return fail(DM_ERR_INVALID_ARG, "plan buffer too small");
    std::memcpy(buf, v.data(), sizeof(int32_t) * v.size());
    return DM_OK;
}

}  // extern "C"

// ------------------------------------------------------------- enumerate

namespace dm {

// Plan a pattern against a data graph with the options' motif subset.
dm_status plan_for(const dm_datagraph* dg, const NormPattern& p, const dm_plan_opts* opts, Plan* plan) {
    uint32_t avail = dg->motif_bits;
    if (opts && opts->motif_mask) {
        uint32_t want = motif_bits_from_mask(opts->motif_mask);
        avail &= want;
    }
    // the plan depends on the pattern's edges, the motifs and the tables'
    // statistics only
    std::string key;
    key.reserve(64 + 8 * p.edges.size());
    auto put = [&](const void* x, size_t n) { key.append((const char*)x, n); };
    put(&p.k, sizeof p.k);
    put(&avail, sizeof avail);
    put(&dg->stats.n_vertices, sizeof dg->stats.n_vertices);
    put(dg->stats.rows, sizeof dg->stats.rows);
    put(&dg->stats.avg_degree, sizeof dg->stats.avg_degree);
    for (auto& e : p.edges) put(&e, sizeof e);
    dm_context* ctx = dg->ctx;
    if (ctx->plans.get(key, plan)) return DM_OK;
    std::string err;
    dm_status st = plan_pattern(p, 0, avail, &dg->stats, plan, &err);
    if (st != DM_OK) return fail(st, err);
    // The decomposition takes the largest motif that fits first (Sec. III-C),
    // which is not always the cheapest (a 7-path through a 3x3 grid filtered
    // by chords; paths where a claw fits a tree-like pattern better): plan
    // again without the end-keyed motifs and without the longer paths, and
    // keep the plan with the least estimated table work.
    uint32_t ends = 0, paths = 0;
    for (int m = 0; m < kNumMotifs; m++) {
        const MotifInfo& mi = motif_info(m);
        if (mi.ends_only) ends |= 1u << m;
        if (!mi.general && !mi.cycle && mi.size >= 3) paths |= 1u << m;
    }
    for (uint32_t drop : {ends, paths}) {
        if (!(avail & drop) || (avail & ~drop) == avail) continue;
        Plan alt;
        if (plan_pattern(p, 0, avail & ~drop, &dg->stats, &alt, &err) == DM_OK && alt.est_cost < plan->est_cost)
            *plan = std::move(alt);
    }
    plan->cache_key = key;
    ctx->plans.put(std::move(key), *plan);
    return DM_OK;
}

RunOptions run_options(const dm_plan_opts* opts, int64_t cap) {
    RunOptions o;
    if (opts) {
        o.block = opts->block_threads;
        o.mode = opts->output_mode;
        o.sync_each_step = opts->sync_each_step != 0;
        o.mem_budget = opts->mem_budget;
        o.profile = opts->profile != 0;
        o.initial_rows = opts->initial_rows;
        o.root_begin = opts->root_begin;
        o.root_end = opts->root_end;
        o.induced = opts->induced != 0;
        o.score = opts->score != 0;
        o.result_limit = opts->result_mb > 0 ? (int64_t)opts->result_mb << 20 : 0;
        o.wait_limit_us = opts->wait_limit_us;
    }
    o.cap = cap;
    return o;
}

// Patterns with more vertices than the data graph, or an empty data graph:
// an empty result without device work.
dm_result* empty_result(dm_context* ctx, int32_t k, int32_t mode) {
    auto* r = new dm_result();
    r->ctx = ctx;
    r->width = k;
    r->stream = ctx->stream;
    r->mode = mode;
    return r;
}

// Layout costs default to zero: allocate zero arrays the first time a scored
// run needs them.
dm_status ensure_costs(dm_datagraph* dg) {
    if (dg->vcost && dg->ecost) return DM_OK;
    hipStream_t s = dg->ctx->stream;
    if (!dg->vcost) {
        DM_TRY(dev_alloc(dg->ctx, (void**)&dg->vcost, sizeof(uint32_t) * (size_t)std::max(dg->n, 1), s));
        DM_HIP(launch_fill_i32((int32_t*)dg->vcost, 0, std::max(dg->n, 1), s));
    }
    if (!dg->ecost) {
        DM_TRY(dev_alloc(dg->ctx, (void**)&dg->ecost, sizeof(uint32_t) * (size_t)std::max<int64_t>(dg->nnz, 1), s));
        DM_HIP(launch_fill_i32((int32_t*)dg->ecost, 0, std::max<int64_t>(dg->nnz, 1), s));
    }
    return DM_OK;
}

dm_status enumerate_one(dm_datagraph* dg, Workspace& ws, const dm_graph_desc* gp, int64_t cap,
                        const dm_plan_opts* opts, dm_result** out) {
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    NormPattern p;
    std::string err;
    dm_status st = normalize_pattern(gp, &p, &err);
    if (st != DM_OK) return fail(st, err);
    const int32_t mode = opts ? opts->output_mode : DM_OUT_TABLE;
    if (mode != DM_OUT_TABLE && mode != DM_OUT_COUNT_HASH) return fail(DM_ERR_INVALID_ARG, "bad output mode");
    if (opts && opts->block_threads != 0 && opts->block_threads != 64 && opts->block_threads != 128 &&
        opts->block_threads != 256)
        return fail(DM_ERR_INVALID_ARG, "block_threads must be 0, 64, 128 or 256");
    if (p.k > dg->n) {
        *out = empty_result(dg->ctx, p.k, mode);
        (*out)->stream = ws.stream;
        return DM_OK;
    }
    Plan plan;
    DM_TRY(plan_for(dg, p, opts, &plan));
    auto t1 = std::chrono::steady_clock::now();
    RunOptions ro = run_options(opts, cap);
    if (ro.score && mode == DM_OUT_TABLE) DM_TRY(ensure_costs(dg));
    RunOutput o;
    DM_TRY(run_plan_chunked(dg->ctx, ws, dg, plan, ro, &o));
    auto* r = new dm_result();
    r->ctx = dg->ctx;
    r->width = p.k;
    r->stream = ws.stream;
    r->mode = mode;
    r->total = o.rows;
    if (mode == DM_OUT_COUNT_HASH) {
        r->rows = 0;
        r->hsum = o.hsum;
        r->hxor = o.hxor;
    } else {
        r->rows = o.sorted_rows;
        r->data = o.sorted;
        r->costs = o.costs;
    }
    r->stats = o.stats;
    r->stats.plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    *out = r;
    return DM_OK;
}

}  // namespace dm

extern "C" {

dm_status dm_estimate(dm_datagraph* dg, const dm_graph_desc* gp, const dm_plan_opts* opts, int64_t* peak_bytes,
                      int64_t* est_rows) {
    if (!dg || !gp) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    NormPattern p;
    std::string err;
    dm_status st = normalize_pattern(gp, &p, &err);
    if (st != DM_OK) return fail(st, err);
    Plan plan;
    DM_TRY(plan_for(dg, p, opts, &plan));
    if (peak_bytes) *peak_bytes = (int64_t)std::min(plan.est_peak_rows_cols * 4.0, 9.0e18);
    if (est_rows) *est_rows = (int64_t)std::min(plan.est_final_rows, 9.0e18);
    return DM_OK;
}

dm_status dm_enumerate(dm_datagraph* dg, const dm_graph_desc* gp, int64_t max_embeddings, const dm_plan_opts* opts,
                       dm_result** out) {
    if (!dg || !gp || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    if (__atomic_load_n(dg->ctx->cancel, __ATOMIC_SEQ_CST)) return fail(DM_ERR_CANCELLED, "context is cancelled");
    DM_HIP(hipSetDevice(dg->ctx->device));
    return enumerate_one(dg, dg->ctx->ws, gp, max_embeddings, opts, out);
}

int64_t dm_result_rows(const dm_result* r) { return r ? r->rows : 0; }
int64_t dm_result_total(const dm_result* r) { return r ? r->total : 0; }
int32_t dm_result_width(const dm_result* r) { return r ? r->width : 0; }
const int32_t* dm_result_device_data(const dm_result* r) { return (r && r->rows > 0) ? r->data : nullptr; }

dm_status dm_result_hash(const dm_result* r, uint64_t* hash_sum, uint64_t* hash_xor) {
    if (!r) return fail(DM_ERR_INVALID_ARG, "NULL result");
    if (r->mode != DM_OUT_COUNT_HASH) return fail(DM_ERR_INVALID_ARG, "result is not in count+hash mode");
    if (hash_sum) *hash_sum = r->hsum;
    if (hash_xor) *hash_xor = r->hxor;
    return DM_OK;
}

dm_status dm_result_copy_to_host(const dm_result* r, int32_t* dst, int64_t max_rows) {
    if (!r || (!dst && max_rows > 0)) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    int64_t n = std::min(max_rows, r->rows);
    if (n <= 0) return DM_OK;
    DM_HIP(hipSetDevice(r->ctx->device));
    DM_HIP(hipMemcpyAsync(dst, r->data, sizeof(int32_t) * (size_t)n * r->width, hipMemcpyDeviceToHost, r->stream));
    DM_HIP(hipStreamSynchronize(r->stream));
    return DM_OK;
}

dm_status dm_result_copy_to_device(const dm_result* r, int32_t* dst, int64_t max_rows, void* hip_stream) {
    if (!r || (!dst && max_rows > 0)) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    int64_t n = std::min(max_rows, r->rows);
    if (n <= 0) return DM_OK;
    DM_HIP(hipSetDevice(r->ctx->device));
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : r->stream;
    if (s != r->stream) {
        hipEvent_t e;
        DM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        DM_HIP(hipEventRecord(e, r->stream));
        DM_HIP(hipStreamWaitEvent(s, e, 0));
        (void)hipEventDestroy(e);
    }
    DM_HIP(hipMemcpyAsync(dst, r->data, sizeof(int32_t) * (size_t)n * r->width, hipMemcpyDeviceToDevice, s));
    DM_HIP(hipStreamSynchronize(s));
    return DM_OK;
}

dm_status dm_result_stats(const dm_result* r, dm_run_stats* out) {
    if (!r || !out) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = r->stats;
    return DM_OK;
}

dm_status dm_result_summaries(dm_result* const* rs, int32_t n, dm_result_summary* out) {
    if (n < 0 || (n > 0 && (!rs || !out))) return fail(DM_ERR_INVALID_ARG, "NULL argument or negative count");
    for (int32_t i = 0; i < n; i++) {
        const dm_result* r = rs[i];
        if (!r) return fail(DM_ERR_INVALID_ARG, "NULL result handle");
        dm_result_summary& o = out[i];
        o.total = r->total;
        o.rows = r->rows;
        o.join_ms = r->stats.join_ms;
        o.sort_ms = r->stats.sort_ms;
        o.join_bytes = r->stats.join_bytes;
        o.sort_bytes = r->stats.sort_bytes;
        o.join_launches = r->stats.join_launches;
        o.sort_launches = r->stats.sort_launches;
    }
    return DM_OK;
}

void dm_result_free_many(dm_result* const* rs, int32_t n) {
    if (!rs) return;
    for (int32_t i = 0; i < n; i++) dm_result_free(rs[i]);
}

void dm_result_free(dm_result* r) {
    if (!r) return;
    if (r->block) {
        r->block.reset();
    } else if (r->data) {
        (void)hipSetDevice(r->ctx->device);
        dev_free(r->ctx, r->data, r->stream);
    }
    if (r->costs) {
        (void)hipSetDevice(r->ctx->device);
        dev_free(r->ctx, r->costs, r->stream);
    }
    delete r;
}

const uint64_t* dm_result_device_costs(const dm_result* r) { return (r && r->rows > 0) ? r->costs : nullptr; }

dm_status dm_result_copy_costs(const dm_result* r, uint64_t* dst, int64_t max_rows) {
    if (!r || (!dst && max_rows > 0)) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    if (!r->costs && r->rows > 0) return fail(DM_ERR_INVALID_ARG, "result was not scored");
    const int64_t n = std::min<int64_t>(max_rows, r->rows);
    if (n <= 0) return DM_OK;
    DM_HIP(hipSetDevice(r->ctx->device));
    DM_HIP(hipMemcpyAsync(dst, r->costs, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost, r->stream));
    DM_HIP(hipStreamSynchronize(r->stream));
    return DM_OK;
}

}  // extern "C"
