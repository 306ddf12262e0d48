// Batched and served forms of Algorithm 1 over one resident data graph.
//
// Batched: every pattern is decomposed on the host, then all join steps of
// all patterns run in ONE persistent kernel launch (device-side stage
// counters and per-(pattern, step) tile tickets, see batch_kernel), followed
// by one launch per sort tier that canonicalizes every pattern's table.
// Patterns whose first-attempt table capacity overflowed are re-run alone
// with exact sizing.
//
// Served: a request loop keeps the data graph resident, admits queries by
// their predicted intermediate-table memory, and runs admitted queries as
// continuous batches on several streams, so work of queries that arrive
// while others are on the GPU overlaps on the device.
#include <algorithm>
#include <functional>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "host_pool.hpp"
#include "runtime.hpp"

using namespace dm;

namespace {

constexpr int kBatchMaxCols = 127;   // widest input table the persistent kernel stages in LDS
// Patterns whose predicted peak tables (rows x columns, input + output of a
// step) pass this run through the per-step launches instead of the
// persistent kernel.
constexpr double kBatchLargeValues = 16.0 * 1024 * 1024;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tuning overrides (DMOTIF_* environment variables), read per call.
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    const int x = std::atoi(v);
    return x > 0 ? x : dflt;
}

struct DevBlock {
    const dm_context* ctx = nullptr;
    void* p = nullptr;
    hipStream_t s = nullptr;  // stream the free is ordered on
    ~DevBlock() { dev_free(ctx, p, s); }
};

struct Item {
    int32_t idx;       // position in the caller's array
    int32_t k;
    int64_t cap = -1;  // max embeddings
    Plan plan;
    std::vector<StepDesc> steps;
    int64_t out_rows = 0;  // rows of its sorted result
    // root range [r0, r1) of the identity table: a capped item starts with the
    // lowest roots expected to hold the cap (grouped-by-root tables make that
    // prefix the start of the canonical order)
    int32_t r0 = 0, r1 = 0;
    // control-arena / result-block offsets (bytes)
    size_t off_counts = 0, off_flags = 0, off_hash = 0, off_res = 0;
};

}  // namespace

namespace dm {

// Run a set of already-validated patterns as one batch on workspace `ws`.
// results[i] receives item i's result (owned by the caller).
//
// One persistent launch runs every pattern's steps; step tables live in the
// workspace's device heap, each cut when its step is published with exactly
// the candidate bound of rows.  After one readback of the counts, the
// result block is allocated at its exact size and the sort runs.
static dm_status run_batch(dm_datagraph* dg, Workspace& ws, std::vector<Item>& items, const dm_plan_opts* opts,
                           std::vector<dm_result*>& results) {
    dm_context* ctx = dg->ctx;
    hipStream_t s = ws.stream;
    const int32_t nv = dg->n;
    const int nb = (int)items.size();
    const bool hash_mode = opts && opts->output_mode == DM_OUT_COUNT_HASH;
    const bool profile = opts && opts->profile;
    const bool timing = std::getenv("DMOTIF_BATCH_TIMING") != nullptr;
    const int64_t row_limit = opts && opts->initial_rows > 0 ? opts->initial_rows : 0;
    const int64_t budget = opts && opts->mem_budget > 0 ? opts->mem_budget : (int64_t)48 << 30;
    results.assign(nb, nullptr);
    if (nb == 0) return DM_OK;
    auto ms_since = [](std::chrono::steady_clock::time_point a) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
    };
    const auto t0 = std::chrono::steady_clock::now();

    // ---- step-0 tables are reserved here; every later table on the device
    int total_steps = 0, cmax = 1, max_k = 1, max_wp = 1;
    for (auto& it : items)
        for (auto& d : it.steps) cmax = std::max(cmax, (int)d.c_in);
    // the tuned launch shape when this batch's widest step fits it, else the defaults
    const bool tuned = dg->batch_block > 0 && cmax <= dg->batch_max_cols;
    const int block = batch_block_for(cmax, tuned ? dg->batch_block : 0);
    const int grid = batch_grid_for(block, cmax, tuned && block == dg->batch_block ? dg->batch_grid : 0);
    int64_t heap0 = 0, words0 = 0;
    std::vector<int64_t> h_off(nb), w_off(nb), rows0(nb);
    for (int p = 0; p < nb; p++) {
        Item& it = items[p];
        const StepDesc& d0 = it.steps[0];
        const int32_t nr = it.r1 - it.r0;
        int64_t r = 0;
        if (!(hash_mode && it.steps.size() == 1))
            r = d0.motif >= 0 ? dg->table_dev(d0.motif, d0.key_pos).rows : (int64_t)nr;
        if (row_limit > 0) r = std::min(r, row_limit);
        rows0[p] = r;
        h_off[p] = heap0;
        heap0 += (r * (d0.c_in + (d0.motif >= 0 ? d0.n_new : 0)) + 63) & ~(int64_t)63;
        w_off[p] = words0;
        words0 += (nr + block - 1) / block + 2;
        total_steps += (int)it.steps.size();
        for (auto& d : it.steps) cmax = std::max(cmax, (int)d.c_in);
        max_k = std::max(max_k, it.k);
    }
    // first heap: 1 GiB (DMOTIF_BATCH_HEAP_MB overrides), within the budget;
    // it grows when a batch does not fit
    const int64_t budget_elems = budget / 4;
    const int64_t first_heap = (int64_t)env_int("DMOTIF_BATCH_HEAP_MB", 1024) << 18;
    DM_TRY(ws.ensure_heap(std::min<int64_t>(std::max<int64_t>(ws.heap_elems, first_heap), budget_elems),
                          2 * heap0, 2 * words0));
    const uint32_t epoch = ws.next_heap_epoch();
    if (epoch == 0) return fail(DM_ERR_DEVICE, "look-back word reset failed");

    // ---- control arena: [counts, flags, hash per item | misc | tops] [jobs] [ctl | first | nsteps | args]
    size_t arena = 0;
    for (auto& it : items) {
        it.off_counts = arena;
        arena = align256(arena + sizeof(int64_t) * (it.steps.size() + 2));
        it.off_flags = arena;
        arena = align256(arena + sizeof(int32_t) * (it.steps.size() + 2));
        it.off_hash = arena;
        arena = align256(arena + sizeof(uint64_t) * 4);
    }
    // finished, sort counters (spill_n[2], max_chunks, dup), abort word, tiles done
    const size_t off_misc = arena;
    arena = align256(arena + 64);
    const size_t off_diag = arena;  // the record of a wait that gave up
    arena = align256(arena + sizeof(WaitDiag));
    const size_t off_fail = arena;
    arena = align256(arena + sizeof(int32_t) * nb);
    const size_t off_tops = arena;  // heap top, words top
    arena = align256(arena + 2 * sizeof(unsigned long long));
    const size_t zero_end = arena;
    const size_t off_jobs = arena;
    arena = align256(arena + sizeof(SortJob) * nb);
    const size_t back_end = arena;
    const size_t off_ctl = arena;
    arena = align256(arena + sizeof(BatchCtl) * nb);
    const size_t off_first = arena;
    arena = align256(arena + sizeof(int32_t) * nb);
    const size_t off_nsteps = arena;
    arena = align256(arena + sizeof(int32_t) * nb);
    const size_t off_args = arena;
    arena = align256(arena + sizeof(EjfArgs) * total_steps);

    char* A = nullptr;
    DM_TRY(dev_alloc(ctx, (void**)&A, arena, s));
    std::unique_ptr<DevBlock> arena_guard(new DevBlock{ctx, A, s});

    // ---- host staging of sort jobs, controllers and argument blocks, built
    // in the workspace's pinned buffer so the upload is an asynchronous DMA
    // (from pageable memory it would first be copied and waited for)
    const size_t host_size = arena - off_jobs;
    DM_TRY(ws.ensure_stage(std::max(host_size, back_end)));
    char* host = ws.stage_h;
    std::memset(host, 0, host_size);
    SortJob* jobs = (SortJob*)(host + (off_jobs - off_jobs));
    BatchCtl* ctl = (BatchCtl*)(host + (off_ctl - off_jobs));
    int32_t* first = (int32_t*)(host + (off_first - off_jobs));
    int32_t* nsteps = (int32_t*)(host + (off_nsteps - off_jobs));
    EjfArgs* args = (EjfArgs*)(host + (off_args - off_jobs));
    int a_i = 0;
    const GraphDev g = dg->graph_dev();
    for (int p = 0; p < nb; p++) {
        Item& it = items[p];
        const int ns = (int)it.steps.size();
        first[p] = a_i;
        nsteps[p] = ns;
        const int32_t nr = it.r1 - it.r0;
        ctl[p].n_in[0] = nr;
        ctl[p].ntiles[0] = (nr + block - 1) / block;
        int64_t* counts = (int64_t*)(A + it.off_counts);
        int32_t* flags = (int32_t*)(A + it.off_flags);
        for (int i = 0; i < ns; i++) {
            EjfArgs& a = args[a_i++];
            std::memset(&a, 0, sizeof a);
            a.st = it.steps[i];
            if (a.st.motif >= 0) a.tbl = dg->table_dev_step(a.st);
            a.g = g;
            a.n_in = &counts[i];
            a.id_begin = it.r0;
            a.id_count = nr;
            a.n_out = &counts[i + 1];
            a.overflow = &flags[i];
            a.epoch = epoch;
            a.ticket = nullptr;
            a.mode = (hash_mode && i == ns - 1) ? EJF_HASH : EJF_WRITE;
            a.hash_acc = (uint64_t*)(A + it.off_hash);
            a.induced = opts && opts->induced ? 1 : 0;
            a.w = wait_ctl(ctx, (uint32_t*)(A + off_misc) + 5, (WaitDiag*)(A + off_diag),
                           opts ? opts->wait_limit_us : 0);
            a.diag_pattern = it.idx;
            a.diag_step = i;
            for (int c = 0; c < it.k; c++) a.pv[c] = (uint8_t)std::max(it.plan.pv_of[c], 0);
            if (i + 1 < ns && !(hash_mode && i + 1 == ns - 1)) {
                const StepDesc& nx = it.steps[i + 1];
                a.next_cand = (int64_t*)(A + off_ctl + sizeof(BatchCtl) * p + offsetof(BatchCtl, cand)) + (i + 1);
                a.next_key_col = nx.motif >= 0 ? nx.key_col : -1;
                a.next_offs = nx.motif >= 0 ? dg->table_dev(nx.motif, nx.key_pos).offs : nullptr;
            }
            if (i == 0) {
                // identity input; output and look-back words reserved above
                a.in = nullptr;
                a.in_cap = nr;
                a.out = ws.heap + h_off[p];
                a.out_stride = std::max<int64_t>(rows0[p], 1);
                a.out_cap = rows0[p];
                a.status = ws.heap_words + w_off[p];
            }
        }
        SortJob& j = jobs[p];
        j.n_in = &counts[ns];
        j.k = it.k;
        sort_pack_layout(it.k, nv, &j);
        max_wp = std::max(max_wp, j.wp);
        for (int c = 0; c < it.k; c++) j.perm[c] = (uint8_t)it.plan.col_of[c];
    }
    int32_t* misc = (int32_t*)(A + off_misc);
    unsigned long long tops[2] = {(unsigned long long)heap0, (unsigned long long)words0};

    DM_HIP(launch_fill_u64((uint64_t*)A, 0, (int64_t)(zero_end / 8), s));
    DM_HIP(hipMemcpyAsync(A + off_tops, tops, sizeof tops, hipMemcpyHostToDevice, s));
    DM_HIP(hipMemcpyAsync(A + off_jobs, host, host_size, hipMemcpyHostToDevice, s));

    hipEvent_t ev[6];
    for (auto& e : ev) DM_HIP(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t* e;
        ~EvGuard() {
            for (int i = 0; i < 6; i++) (void)hipEventDestroy(e[i]);
        }
    } evg{ev};

    BatchDev bd;
    std::memset(&bd, 0, sizeof bd);
    bd.args = (EjfArgs*)(A + off_args);
    bd.first = (const int32_t*)(A + off_first);
    bd.nsteps = (const int32_t*)(A + off_nsteps);
    bd.ctl = (BatchCtl*)(A + off_ctl);
    bd.finished = &misc[0];
    bd.heap_fail = (int32_t*)(A + off_fail);
    bd.jobs = hash_mode ? nullptr : (SortJob*)(A + off_jobs);
    bd.heap = ws.heap;
    bd.heap_cap = std::max(std::min(ws.heap_elems, budget_elems), heap0);
    bd.heap_top = (unsigned long long*)(A + off_tops);
    bd.words = ws.heap_words;
    bd.words_cap = ws.heap_words_cap;
    bd.words_top = (unsigned long long*)(A + off_tops) + 1;
    bd.row_limit = row_limit;
    bd.n_patterns = nb;
    bd.max_backoff = tuned && dg->batch_backoff > 0 ? dg->batch_backoff : 15;
    bd.w = wait_ctl(ctx, (uint32_t*)&misc[5], (WaitDiag*)(A + off_diag), opts ? opts->wait_limit_us : 0);
    bd.tiles_done = (uint32_t*)&misc[6];
    const double t_stage = ms_since(t0);
    DM_HIP(hipEventRecord(ev[0], s));
    bool wide = false;
    for (auto& it : items)
        for (auto& d : it.steps) wide |= d.motif >= 0 && d.n_new > kNarrowNew;
    DM_HIP(launch_batch(bd, block, cmax, wide, grid, s));
    DM_HIP(hipEventRecord(ev[1], s));

    // ---- readback 1: counts, flags, hashes, failures, heap use, sort jobs
    // (through the pinned buffer, queued after the upload that read it)
    DM_HIP(hipMemcpyAsync(ws.stage_h, A, back_end, hipMemcpyDeviceToHost, s));
    DM_HIP(hipStreamSynchronize(s));
    std::vector<char> back(ws.stage_h, ws.stage_h + back_end);
    const double t_join = ms_since(t0);
    auto hb = [&](size_t off) { return back.data() + off; };
    const int32_t* hmisc = (const int32_t*)hb(off_misc);
    DM_TRY(check_abort((uint32_t)hmisc[5], *(const WaitDiag*)hb(off_diag), "persistent join"));
    if (hmisc[0] != nb) return fail(DM_ERR_INTERNAL, "persistent kernel retired " + std::to_string(hmisc[0]) +
                                                         " of " + std::to_string(nb) + " patterns");
    const int32_t* hfail = (const int32_t*)hb(off_fail);
    const unsigned long long* htops = (const unsigned long long*)hb(off_tops);
    if (const char* trace = std::getenv("DMOTIF_BATCH_TRACE")) {
        // per-pattern stage timeline (device wall clock at each step's publication)
        std::vector<BatchCtl> hc(nb);
        DM_HIP(hipMemcpy(hc.data(), A + off_ctl, sizeof(BatchCtl) * nb, hipMemcpyDeviceToHost));
        int khz = 100000;
        (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device);
        if (FILE* f = std::fopen(trace, "a")) {
            int64_t tmin = INT64_MAX;
            for (int p = 0; p < nb; p++) tmin = std::min(tmin, hc[p].t_pub[0]);
            for (int p = 0; p < nb; p++) {
                const int ns = (int)items[p].steps.size();
                const int64_t* counts = (const int64_t*)hb(items[p].off_counts);
                std::fprintf(f, "{\"pattern\": %d, \"k\": %d, \"steps\": [", items[p].idx, items[p].k);
                for (int i = 0; i <= ns; i++) {
                    const double us = hc[p].t_pub[i] ? 1e3 * (double)(hc[p].t_pub[i] - tmin) / khz : -1.0;
                    std::fprintf(f, "%s[%.1f, %lld, %d]", i ? ", " : "", us, (long long)counts[i],
                                 i < ns ? hc[p].ntiles[i] : 0);
                }
                std::fprintf(f, "]}\n");
            }
            std::fclose(f);
        }
    }

    // ---- classify: done in the batch, or redone (overflow, short prefix, no heap room)
    std::vector<char> redo(nb, 0), grow(nb, 0);
    std::vector<int64_t> n_final(nb, 0);
    size_t resb = 0;
    int64_t max_rows = 1;
    int n_grow = 0;
    SortJob* hjobs = (SortJob*)hb(off_jobs);
    for (int p = 0; p < nb; p++) {
        Item& it = items[p];
        const int ns = (int)it.steps.size();
        const int64_t* counts = (const int64_t*)hb(it.off_counts);
        const int32_t* flags = (const int32_t*)hb(it.off_flags);
        const uint64_t* hash = (const uint64_t*)hb(it.off_hash);
        bool over = false;
        for (int i = 0; i < ns; i++) over |= flags[i] != 0;
        n_final[p] = hash_mode ? (int64_t)hash[0] : counts[ns];
        // a capped item whose root prefix held fewer rows than the cap
        const bool partial = !hash_mode && !over && it.r1 < nv && it.cap >= 0 && n_final[p] < it.cap;
        if (hfail[p]) {
            grow[p] = 1;
            n_grow++;
        } else if (over || partial) {
            redo[p] = 1;
        }
        SortJob& j = hjobs[p];
        if (hash_mode || grow[p] || redo[p] || n_final[p] == 0) {
            j.in_cap = 0;  // nothing to sort for this job
            j.out = nullptr;
            j.out_rows = 0;
            it.out_rows = 0;
            continue;
        }
        it.out_rows = it.cap >= 0 ? std::min<int64_t>(it.cap, n_final[p]) : n_final[p];
        if (opts && opts->result_mb > 0 && it.out_rows * 4 * (int64_t)it.k > ((int64_t)opts->result_mb << 20))
            return fail(DM_ERR_BUDGET_EXCEEDED, "pattern " + std::to_string(it.idx) + ": result of " +
                                                    std::to_string(it.out_rows) + " rows exceeds result_mb");
        it.off_res = resb;
        resb = align256(resb + sizeof(int32_t) * (size_t)std::max<int64_t>(it.out_rows * it.k, 1));
        max_rows = std::max(max_rows, n_final[p]);
    }

    // ---- sort into the exact-size result block
    std::shared_ptr<DevBlock> res_block;
    char* R = nullptr;
    float ms_join = 0, ms_sort = 0;
    (void)hipEventElapsedTime(&ms_join, ev[0], ev[1]);
    double t_ralloc = 0;
    if (!hash_mode && resb > 0) {
        const auto ta = std::chrono::steady_clock::now();
        DM_TRY(dev_alloc(ctx, (void**)&R, resb, s));
        t_ralloc = ms_since(ta);
        res_block.reset(new DevBlock{ctx, R, s});
        for (int p = 0; p < nb; p++) {
            if (items[p].out_rows > 0) hjobs[p].out = (int32_t*)(R + items[p].off_res);
            hjobs[p].out_rows = items[p].out_rows;
        }
        DM_HIP(hipMemcpyAsync(A + off_jobs, hjobs, sizeof(SortJob) * nb, hipMemcpyHostToDevice, s));
        DM_HIP(hipEventRecord(ev[2], s));
        bool merged = false;
        DM_TRY(enqueue_sort(ctx, ws, (const SortJob*)(A + off_jobs), nb, nv, 0, max_rows, max_wp, &misc[1],
                            (const uint32_t*)&misc[5], (int32_t*)ws.stage_h, &ev[3], &merged));
        int32_t sc[4];
        DM_HIP(hipMemcpyAsync(sc, &misc[1], sizeof sc, hipMemcpyDeviceToHost, s));
        DM_HIP(hipStreamSynchronize(s));
        if (sc[3] != 0) return fail(DM_ERR_INTERNAL, "duplicate rows reached a canonical table");
        (void)hipEventElapsedTime(&ms_sort, ev[2], ev[3]);
        if (merged) {
            float tm = 0;
            (void)hipEventElapsedTime(&tm, ev[4], ev[5]);
            ms_sort += tm;
        }
    }
    if (timing)
        std::fprintf(stderr,
                     "[batch] %d patterns | heap %.1f MB used of %.1f MB, words %llu | results %.1f MB | stage %.2f ms, "
                     "join+readback %.2f ms, sort+readback %.2f ms (result alloc %.2f ms) | join %.2f ms, sort %.2f ms | "
                     "redo %d, grow %d\n",
                     nb, 4e-6 * (double)htops[0], 4e-6 * (double)ws.heap_elems, (unsigned long long)htops[1],
                     resb / 1e6, t_stage, t_join - t_stage, ms_since(t0) - t_join, t_ralloc, ms_join, ms_sort,
                     (int)std::count(redo.begin(), redo.end(), 1), n_grow);

    // ---- patterns whose tables did not fit: a larger heap, then one more batch
    std::vector<dm_result*> regrown;
    std::vector<int> grow_idx;
    if (n_grow > 0) {
        const int64_t used = (int64_t)htops[0];
        const int64_t want = std::min<int64_t>(std::max<int64_t>(4 * bd.heap_cap, 2 * used), budget_elems);
        std::vector<Item> sub;
        for (int p = 0; p < nb; p++)
            if (grow[p]) {
                if (want > bd.heap_cap) {
                    sub.push_back(items[p]);
                    grow_idx.push_back(p);
                } else {
                    redo[p] = 1;  // the heap is at the memory budget: root-range chunks instead
                }
            }
        if (!sub.empty()) {
            DM_TRY(ws.ensure_heap(want, 0, 0));
            DM_TRY(run_batch(dg, ws, sub, opts, regrown));
        }
    }

    int64_t all_bytes = 0;
    std::vector<int64_t> pbytes(nb, 0);
    auto cleanup = [&]() {
        for (auto*& r : results) dm_result_free(r), r = nullptr;
        for (auto*& r : regrown) dm_result_free(r), r = nullptr;
    };
    for (size_t q = 0; q < grow_idx.size(); q++) {
        results[grow_idx[q]] = regrown[q];
        regrown[q] = nullptr;
    }
    for (int p = 0; p < nb; p++) {
        if (results[p]) continue;
        Item& it = items[p];
        const int ns = (int)it.steps.size();
        const int64_t* counts = (const int64_t*)hb(it.off_counts);
        const uint64_t* hash = (const uint64_t*)hb(it.off_hash);
        dm_result* r = nullptr;
        if (redo[p]) {
            // first-attempt capacity too small, a short root prefix, or no
            // heap room within the budget: redo this pattern alone over every
            // root, exact sizes
            RunOptions ro = run_options(opts, it.cap);
            ro.sync_each_step = true;
            RunOutput o;
            dm_status st = run_plan_chunked(ctx, ws, dg, it.plan, ro, &o);
            if (st != DM_OK) {
                cleanup();
                return st;
            }
            r = new dm_result();
            r->ctx = ctx;
            r->width = it.k;
            r->stream = ctx->stream;
            r->mode = hash_mode ? DM_OUT_COUNT_HASH : DM_OUT_TABLE;
            r->total = o.rows;
            if (hash_mode) {
                r->hsum = o.hsum;
                r->hxor = o.hxor;
            } else {
                r->rows = o.sorted_rows;
                r->data = o.sorted;
            }
            r->stats = o.stats;
            r->stats.retries += 1;
        } else {
            r = new dm_result();
            r->ctx = ctx;
            r->width = it.k;
            r->stream = ctx->stream;
            r->mode = hash_mode ? DM_OUT_COUNT_HASH : DM_OUT_TABLE;
            r->total = (it.r1 < nv || it.r0 > 0) ? -1 : n_final[p];  // a root prefix does not count them all
            if (hash_mode) {
                r->hsum = hash[1];
                r->hxor = hash[2];
            } else {
                r->rows = it.out_rows;
                if (it.out_rows > 0) {
                    r->data = (int32_t*)(R + it.off_res);
                    r->block = res_block;
                }
            }
            r->stats.n_steps = (int32_t)it.plan.steps.size();
            r->stats.chunks = 1;
            int64_t prev_rows = it.r1 - it.r0, bytes = 0;
            int prev_cols = 1;
            for (int i = 0; i < ns; i++) {
                const int64_t rr = (hash_mode && i == ns - 1) ? (int64_t)hash[0] : counts[i + 1];
                if (i < DM_MAX_PATTERN_VERTICES) r->stats.step_rows[i] = rr;
                const int cols = it.steps[i].c_in + it.steps[i].n_new;
                bytes += (i == 0 ? 0 : 4 * (int64_t)prev_cols * prev_rows) +
                         ((hash_mode && i == ns - 1) ? 0 : 4 * (int64_t)cols * rr);
                prev_rows = rr;
                prev_cols = cols;
            }
            r->stats.join_bytes = bytes;
            if (!hash_mode) r->stats.sort_bytes = 8 * (int64_t)it.k * n_final[p];
            r->stats.bytes_moved = r->stats.join_bytes + r->stats.sort_bytes;
            pbytes[p] = bytes;
            all_bytes += bytes;
        }
        results[p] = r;
    }
    // batch-level device times, split by each pattern's share of the bytes so
    // that sums over the batch give the launch totals
    int64_t all_sort = 0;
    for (int p = 0; p < nb; p++)
        if (pbytes[p] > 0) all_sort += results[p]->stats.sort_bytes;
    for (int p = 0; p < nb; p++) {
        dm_result* r = results[p];
        if (pbytes[p] == 0) continue;  // redone or regrown: its own stats
        const double fj = all_bytes > 0 ? (double)pbytes[p] / all_bytes : 1.0 / nb;
        const double fs = all_sort > 0 ? (double)r->stats.sort_bytes / all_sort : 1.0 / nb;
        r->stats.device_ms = fj * ms_join + fs * ms_sort;
        if (profile) {
            r->stats.join_ms = fj * ms_join;
            r->stats.sort_ms = fs * ms_sort;
            r->stats.join_launches = p == 0 ? 1 : 0;
            r->stats.sort_launches = (p == 0 && !hash_mode) ? 3 : 0;
        }
    }
    return DM_OK;
}

// Validate and plan a batch; patterns the persistent kernel cannot hold
// (more than kBatchMaxCols input columns) or with more vertices than the
// data graph are handled apart.
dm_status enumerate_many(dm_datagraph* dg, Workspace& ws, int32_t n, const dm_graph_desc* gps, const int64_t* caps,
                         const dm_plan_opts* opts, dm_result** outs) {
    for (int32_t i = 0; i < n; i++) outs[i] = nullptr;
    const int32_t mode = opts ? opts->output_mode : DM_OUT_TABLE;
    if (mode != DM_OUT_TABLE && mode != DM_OUT_COUNT_HASH) return fail(DM_ERR_INVALID_ARG, "bad output mode");
    const auto t_plan0 = std::chrono::steady_clock::now();
    std::vector<Item> items;
    std::vector<int32_t> solo;
    std::vector<dm_result*> done(n, nullptr);
    auto cleanup = [&]() {
        for (auto*& r : done) dm_result_free(r), r = nullptr;
    };
    // validate and plan every pattern (in parallel on the host workers), then
    // take the results in order so the first failing pattern is reported
    struct Prep {
        dm_status st = DM_OK;
        std::string err;
        int32_t k = 0;
        Plan plan;
    };
    std::vector<Prep> prep(n);
    HostPool::get().parallel_for(n, [&](int i) {
        Prep& q = prep[i];
        NormPattern p;
        std::string err;
        q.st = normalize_pattern(&gps[i], &p, &err);
        if (q.st != DM_OK) {
            q.err = "pattern " + std::to_string(i) + ": " + err;
            return;
        }
        q.k = p.k;
        if (p.k > dg->n) return;
        q.st = plan_for(dg, p, opts, &q.plan);
        if (q.st != DM_OK) q.err = dm_last_error();
    });
    for (int32_t i = 0; i < n; i++) {
        Prep& q = prep[i];
        if (q.st != DM_OK) {
            cleanup();
            return fail(q.st, q.err);
        }
        const int64_t cap = caps ? caps[i] : -1;
        if (q.k > dg->n) {
            done[i] = empty_result(dg->ctx, q.k, mode);
            continue;
        }
        Item it;
        it.idx = i;
        it.k = q.k;
        it.cap = cap;
        it.plan = std::move(q.plan);
        for (auto& ps : it.plan.steps) it.steps.push_back(ps.d);
        if (it.steps.empty()) {
            StepDesc d;
            std::memset(&d, 0, sizeof d);
            d.motif = -1;
            d.c_in = 1;
            it.steps.push_back(d);
        }
        it.r0 = 0;
        it.r1 = dg->n;
        if (cap >= 0 && mode == DM_OUT_TABLE && !it.plan.steps.empty()) {
            // lowest roots expected to hold the cap with a wide margin (roots at
            // the low end may sit on the graph's boundary); a short prefix is
            // redone over every root
            const double per_root = std::max(it.plan.steps.back().est_rows / std::max(dg->n, 1), 1e-9);
            const double roots = std::ceil((8.0 * (double)cap + 256.0) / per_root);
            if (roots < (double)dg->n) it.r1 = std::min<int32_t>(dg->n, std::max<int32_t>(64, (int32_t)roots));
        }
        int cm = 0;
        for (auto& d : it.steps) cm = std::max(cm, (int)d.c_in);
        // a caller's root range and scored runs go through the single-pattern
        // path, and so do patterns predicted to build large tables: the
        // persistent kernel is made for many short chains of small tables
        // (one workgroup per CU), the per-step launches for throughput
        const bool own_path = (opts && opts->root_end > opts->root_begin) || (opts && opts->score && mode == DM_OUT_TABLE);
        const double share = (double)(it.r1 - it.r0) / std::max(dg->n, 1);
        const bool large = it.plan.est_peak_rows_cols * share > kBatchLargeValues;
        if (cm > kBatchMaxCols || (int)it.steps.size() > kMaxSteps || own_path || large) {
            solo.push_back(i);
            continue;
        }
        items.push_back(std::move(it));
    }
    if (std::getenv("DMOTIF_BATCH_TIMING"))
        std::fprintf(stderr, "[batch] validate+plan %d patterns: %.2f ms\n", n,
                     std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_plan0).count());
    std::vector<dm_result*> res;
    dm_status st = run_batch(dg, ws, items, opts, res);
    if (st != DM_OK) {
        cleanup();
        return st;
    }
    for (size_t j = 0; j < items.size(); j++) done[items[j].idx] = res[j];
    if (!solo.empty() && __atomic_load_n(dg->ctx->cancel, __ATOMIC_SEQ_CST)) {
        cleanup();
        return fail(DM_ERR_CANCELLED, "context is cancelled");
    }
    for (int32_t i : solo) {
        st = enumerate_one(dg, ws, &gps[i], caps ? caps[i] : -1, opts, &done[i]);
        if (st != DM_OK) {
            cleanup();
            return st;
        }
    }
    for (int32_t i = 0; i < n; i++) outs[i] = done[i];
    return DM_OK;
}

}  // namespace dm

extern "C" dm_status dm_enumerate_batch(dm_datagraph* dg, int32_t n, const dm_graph_desc* gps, const int64_t* caps,
                                        const dm_plan_opts* opts, dm_result** outs) {
    if (!dg || n < 0 || (n > 0 && (!gps || !outs))) return fail(DM_ERR_INVALID_ARG, "invalid batch arguments");
    DM_HIP(hipSetDevice(dg->ctx->device));
    return enumerate_many(dg, dg->ctx->ws, n, gps, caps, opts, outs);
}

// ------------------------------------------------------------------ motif-set tuning

extern "C" dm_status dm_autotune_motifs(dm_context* ctx, const dm_graph_desc* gd, int32_t n_sample,
                                        const dm_graph_desc* sample, const uint32_t* candidates,
                                        int32_t n_candidates, int32_t reps, uint32_t* best_mask,
                                        double* ms_per_candidate) {
    if (!ctx || !gd || !best_mask || n_sample <= 0 || !sample || n_candidates <= 0 || !candidates || reps <= 0)
        return fail(DM_ERR_INVALID_ARG, "invalid tuning arguments");
    DM_HIP(hipSetDevice(ctx->device));
    dm_plan_opts opts;
    std::memset(&opts, 0, sizeof opts);
    opts.output_mode = DM_OUT_COUNT_HASH;
    std::vector<dm_result*> outs((size_t)n_sample, nullptr);
    double best = 1e300;
    int best_i = -1;
    for (int32_t c = 0; c < n_candidates; c++) {
        // the planner may use every table the data graph holds
        opts.motif_mask = candidates[c] == DM_MOTIF_M2_ONLY ? DM_MOTIF_M2_ONLY : 0;
        std::vector<double> t;
        for (int32_t r = 0; r < reps; r++) {
            const auto t0 = std::chrono::steady_clock::now();
            dm_datagraph* dg = nullptr;
            DM_TRY(dm_datagraph_build(ctx, gd, candidates[c], &dg));
            dm_status st = enumerate_many(dg, ctx->ws, n_sample, sample, nullptr, &opts, outs.data());
            for (auto*& o : outs) dm_result_free(o), o = nullptr;
            (void)dm_datagraph_free(dg);
            if (st != DM_OK) return st;
            t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        std::sort(t.begin(), t.end());
        const double med = t[t.size() / 2];
        if (ms_per_candidate) ms_per_candidate[c] = med;
        if (med < best) {
            best = med;
            best_i = c;
        }
    }
    *best_mask = candidates[best_i];
    return DM_OK;
}

// ------------------------------------------------------------------ launch-shape tuning

extern "C" dm_status dm_autotune_batch(dm_datagraph* dg, int32_t n_sample, const dm_graph_desc* sample,
                                       int32_t reps, dm_batch_tuning* best, dm_batch_tuning* tried,
                                       int32_t tried_cap, int32_t* n_tried) {
    if (!dg || n_sample <= 0 || !sample || reps <= 0 || !best || (tried_cap > 0 && !tried))
        return fail(DM_ERR_INVALID_ARG, "invalid tuning arguments");
    DM_HIP(hipSetDevice(dg->ctx->device));
    // the sample's widest step decides which block sizes can run it
    int cmax = 1;
    for (int32_t i = 0; i < n_sample; i++) {
        NormPattern p;
        std::string err;
        dm_status st = normalize_pattern(&sample[i], &p, &err);
        if (st != DM_OK) return fail(st, "sample pattern " + std::to_string(i) + ": " + err);
        if (p.k > dg->n) continue;
        Plan plan;
        DM_TRY(plan_for(dg, p, nullptr, &plan));
        for (auto& s : plan.steps) cmax = std::max(cmax, (int)s.d.c_in);
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dg->ctx->device);
    const int widest = batch_block_for(cmax, 0);
    std::vector<dm_batch_tuning> cand;
    for (int block : {256, 128, 64}) {
        if (block > widest) continue;
        for (double per_cu : {0.75, 1.0, 1.25, 1.5})
            for (int backoff : {15, 7, 31}) {
                dm_batch_tuning c{};
                c.block_threads = block;
                c.grid = std::max(1, (int)(per_cu * cus * (256 / block)));
                c.backoff = backoff;
                cand.push_back(c);
            }
    }
    const int32_t old_block = dg->batch_block, old_grid = dg->batch_grid, old_backoff = dg->batch_backoff,
                  old_cols = dg->batch_max_cols;
    auto restore = [&]() {
        dg->batch_block = old_block;
        dg->batch_grid = old_grid;
        dg->batch_backoff = old_backoff;
        dg->batch_max_cols = old_cols;
    };
    dm_plan_opts opts;
    std::memset(&opts, 0, sizeof opts);
    opts.output_mode = DM_OUT_COUNT_HASH;
    std::vector<dm_result*> outs((size_t)n_sample, nullptr);
    int best_i = -1;
    int32_t run = 0;
    for (size_t ci = 0; ci < cand.size(); ci++) {
        dm_batch_tuning& c = cand[ci];
        dg->batch_block = c.block_threads;
        dg->batch_grid = c.grid;
        dg->batch_backoff = c.backoff;
        dg->batch_max_cols = cmax;
        std::vector<double> t;
        for (int32_t r = 0; r < reps; r++) {
            const auto t0 = std::chrono::steady_clock::now();
            dm_status st = enumerate_many(dg, dg->ctx->ws, n_sample, sample, nullptr, &opts, outs.data());
            for (auto*& o : outs) dm_result_free(o), o = nullptr;
            if (st != DM_OK) {
                restore();
                return st;
            }
            t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        std::sort(t.begin(), t.end());
        c.ms = t[t.size() / 2];
        if (run < tried_cap) tried[run] = c;
        run++;
        if (best_i < 0 || c.ms < cand[best_i].ms) best_i = (int)ci;
    }
    if (n_tried) *n_tried = run;
    *best = cand[best_i];
    dg->batch_block = best->block_threads;
    dg->batch_grid = best->grid;
    dg->batch_backoff = best->backoff;
    dg->batch_max_cols = cmax;
    return DM_OK;
}

// ------------------------------------------------------------------ server

namespace {

// Queries whose predicted tables stay within this are tiny: consecutive tiny
// queries share one batch of at most kServeTinyBatchBytes predicted tables.
constexpr int64_t kServeTinyBytes = (int64_t)4 << 20;
constexpr int64_t kServeTinyBatchBytes = (int64_t)32 << 20;

struct Request {
    uint64_t ticket = 0;
    int32_t nv = 0;
    std::vector<int32_t> edges;
    int64_t cap = -1;
    int64_t est_bytes = 0;
    bool tiny = false;   // predicted tables within kServeTinyBytes: may share a batch
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
    std::deque<uint64_t> completed;  // finished tickets in completion order (dm_server_wait_any)
    uint64_t next_ticket = 1;
    int32_t inflight = 0;
    bool stopping = false;
};

// Each worker owns one stream + workspace and takes work from the head of
// the queue, so queries start in arrival order and up to n_streams of them
// overlap on the device (one query's host round trips and launch gaps are
// filled by another's kernels).  A tiny query (predicted tables up to
// kServeTinyBytes) takes the tiny ones queued right behind it into the same
// batch (up to max_batch, kServeTinyBatchBytes of predicted tables): one
// persistent launch then runs their short chains together.  Every other
// query runs alone, through the per-step launches, so no query waits inside
// a longer one's batch.  Every query runs within the budget, so the server
// holds at most n_streams x mem_budget of tables.
static void server_worker(dm_server* s, int w) {
    (void)hipSetDevice(s->dg->ctx->device);
    Workspace& ws = *s->ws[w];
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty() && s->stopping) return;
            int64_t batch_bytes = 0;
            while (!s->queue.empty() && (int32_t)batch.size() < s->opts.max_batch) {
                auto& r = s->queue.front();
                if (!batch.empty() && (!r->tiny || batch_bytes + r->est_bytes > kServeTinyBatchBytes)) break;
                batch_bytes += r->est_bytes;
                s->inflight++;
                batch.push_back(r);
                s->queue.pop_front();
                if (!batch.back()->tiny) break;
            }
        }
        std::vector<dm_graph_desc> gps;
        std::vector<int64_t> caps;
        for (auto& r : batch) {
            gps.push_back(dm_graph_desc{r->nv, (int64_t)(r->edges.size() / 2), r->edges.data()});
            caps.push_back(r->cap);
        }
        std::vector<dm_result*> outs(batch.size(), nullptr);
        // each query runs within the server's memory budget
        dm_plan_opts run_opts;
        std::memset(&run_opts, 0, sizeof run_opts);
        run_opts.output_mode = DM_OUT_TABLE;
        run_opts.mem_budget = s->opts.mem_budget;
        run_opts.result_mb = (int32_t)std::min<int64_t>(std::max<int64_t>(s->opts.mem_budget >> 20, 1), INT32_MAX);
        // a query alone takes the plain path (per-step launches); tiny ones share the persistent launch
        dm_status st = (batch.size() == 1 && !batch[0]->tiny)
                           ? enumerate_one(s->dg, ws, &gps[0], caps[0], &run_opts, &outs[0])
                           : enumerate_many(s->dg, ws, (int32_t)batch.size(), gps.data(), caps.data(), &run_opts,
                                            outs.data());
        std::string err = st == DM_OK ? std::string() : std::string(dm_last_error());
        if (st != DM_OK && batch.size() > 1) {
            // isolate the failing request(s): run them one by one
            for (size_t i = 0; i < batch.size(); i++) {
                dm_status si = enumerate_many(s->dg, ws, 1, &gps[i], &caps[i], &run_opts, &outs[i]);
                std::lock_guard<std::mutex> lk(s->mu);
                batch[i]->status = si;
                batch[i]->err = si == DM_OK ? std::string() : std::string(dm_last_error());
            }
        } else {
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto& r : batch) {
                r->status = st;
                r->err = err;
            }
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < batch.size(); i++) {
                auto& r = batch[i];
                // the worker synchronized its stream, so the table is complete;
                // later copies and the free are ordered on the context stream,
                // which outlives the server's own streams
                if (outs[i]) {
                    outs[i]->stream = s->dg->ctx->stream;
                    // a batch's results share one block: its free follows the
                    // context stream too, which outlives the worker streams
                    if (outs[i]->block) static_cast<DevBlock*>(outs[i]->block.get())->s = s->dg->ctx->stream;
                }
                r->result = r->status == DM_OK ? outs[i] : nullptr;
                if (r->status != DM_OK && outs[i]) dm_result_free(outs[i]);
                r->done = true;
                s->completed.push_back(r->ticket);
                s->inflight--;
            }
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
            for (auto& x : s->ws) x->release();
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(DM_ERR_DEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
        auto w = std::make_unique<Workspace>();
        dm_status e = w->init(dg->ctx, st);
        if (e != DM_OK) {
            w->release();
            for (auto& x : s->ws) x->release();
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return e;
        }
        s->ws.push_back(std::move(w));
    }
    dg->servers.fetch_add(1);
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
    // Predicted table bytes.  A capped query is run over the root prefix that
    // should hold 8 x cap rows (as the batch does), so it is predicted over
    // that share of the roots; no query is predicted beyond the budget it
    // runs within.
    int64_t peak = 0, rows = 0;
    if (dm_estimate(s->dg, gp, nullptr, &peak, &rows) == DM_OK) {
        double est = (double)peak;
        const int32_t nv = std::max(s->dg->n, 1);
        if (max_embeddings >= 0 && rows > 0) {
            const double per_root = (double)rows / nv;
            const double roots = (8.0 * (double)max_embeddings + 256.0) / per_root;
            est *= std::min(1.0, std::max(roots, 64.0) / nv);
        }
        r->est_bytes = (int64_t)std::max(1.0, std::min(est, (double)s->opts.mem_budget));
        r->tiny = est <= (double)kServeTinyBytes;
        // refused at admission: a result predicted far beyond the budget it
        // would run within (the prediction can be off by a few times, so
        // only beyond 8x; the rest run and are refused if they pass it)
        const double kept = max_embeddings >= 0 ? std::min((double)max_embeddings, (double)rows) : (double)rows;
        if (kept * 4.0 * p.k > 8.0 * (double)s->opts.mem_budget) {
            r->status = DM_ERR_BUDGET_EXCEEDED;
            r->err = "predicted result of " + std::to_string((int64_t)kept) + " rows exceeds the server's budget";
            r->done = true;
        }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(DM_ERR_CANCELLED, "server is stopping");
    if ((int32_t)s->queue.size() >= s->opts.max_queue) return fail(DM_ERR_BUSY, "server queue is full");
    r->ticket = s->next_ticket++;
    s->live[r->ticket] = r;
    *ticket = r->ticket;
    if (r->done) {
        s->completed.push_back(r->ticket);
        s->cv_done.notify_all();
        return DM_OK;
    }
    s->queue.push_back(r);
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

dm_status dm_server_wait_any(dm_server* s, int32_t timeout_ms, uint64_t* ticket, dm_result** out,
                             dm_status* status) {
    if (!s || !ticket || !out || !status) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    *ticket = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    // tickets already taken by dm_server_wait are passed over
    auto ready = [&] {
        while (!s->completed.empty() && !s->live.count(s->completed.front())) s->completed.pop_front();
        return !s->completed.empty();
    };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return fail(DM_ERR_TIMEOUT, "no request finished");
    }
    const uint64_t t = s->completed.front();
    s->completed.pop_front();
    auto r = s->live[t];
    s->live.erase(t);
    *ticket = t;
    *status = r->status;
    if (r->status == DM_OK) *out = r->result;
    else set_error(r->err);
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
    s->dg->servers.fetch_sub(1);
    delete s;
    return DM_OK;
}

}  // extern "C"
