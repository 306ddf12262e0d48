// Host runtime internals: context, resident data graph, workspaces, results.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "dm_common.hpp"
#include "dm_device.hpp"
#include "host_pool.hpp"

struct dm_context;

namespace dm {

void set_error(const std::string& msg);
dm_status fail(dm_status s, const std::string& msg);
dm_status hip_fail(hipError_t e, const char* what);

#define DM_HIP(call)                                      \
    do {                                                  \
        hipError_t e__ = (call);                          \
        if (e__ != hipSuccess) return hip_fail(e__, #call); \
    } while (0)

#define DM_TRY(call)                     \
    do {                                 \
        dm_status s__ = (call);          \
        if (s__ != DM_OK) return s__;    \
    } while (0)

// Stream-ordered device allocation through the context's allocator (the
// caller's dm_allocator, or the device's default memory pool): every device
// buffer the library holds is taken and returned here.
dm_status dev_alloc(const dm_context* ctx, void** p, size_t bytes, hipStream_t s);
void dev_free(const dm_context* ctx, void* p, hipStream_t s);

// Per-run control block in device memory (counts, flags, hash accumulators).
struct Control {
    int64_t counts[kMaxSteps + 2];
    int32_t overflow[kMaxSteps + 2];
    uint64_t hash[4];
    int32_t sort_counters[6];  // sort tiers: spill_n[2], max_chunks, dup, segments the streaming pass flagged, pad
    uint32_t abort;            // WaitCtl::abort of the run
    uint32_t pad_;
    WaitDiag diag;             // WaitCtl::diag of the run
    int64_t slice_row0;        // first row of a motif table read in place over a root range
};

// Scratch reused across runs of one stream: ping-pong SoA tables, look-back
// words, epoch tickets, spill lists and the control block.
struct Workspace {
    dm_context* ctx = nullptr;  // allocator, cancel word
    hipStream_t stream = nullptr;
    int32_t* buf[2] = {nullptr, nullptr};
    int64_t buf_elems[2] = {0, 0};
    uint64_t* status = nullptr;
    int64_t status_cap = 0;
    uint64_t* tickets = nullptr;  // kEpochs counters
    uint32_t epoch = 0;           // last used epoch (1..kEpochs-1)
    Control* ctrl_d = nullptr;
    Control* ctrl_h = nullptr;    // pinned host mirror
    SegRef* spill = nullptr;      // 2 lists of n_vertices entries (sort tier hand-over)
    int64_t spill_cap = 0;
    uint32_t* spill_bits = nullptr;  // spill_cap epoch words after the lists: segments left to sort
    uint32_t* sort_scratch = nullptr;
    int64_t sort_scratch_elems = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> prof;  // event pairs for per-launch timing
    SortJob* job_d = nullptr;      // one sort job (plain path) and its pinned staging
    SortJob* job_h = nullptr;
    char* stage_h = nullptr;       // pinned host staging for readbacks (grows on demand)
    size_t stage_bytes = 0;
    dm_status ensure_stage(size_t bytes);
    uint64_t* cbuf[2] = {nullptr, nullptr};  // scored runs: cost of each row of buf[i]
    int64_t cbuf_rows[2] = {0, 0};
    dm_status ensure_cbuf(int i, int64_t rows);
    // batched form: device heap of step tables and look-back words (grows on demand)
    int32_t* heap = nullptr;
    int64_t heap_elems = 0;
    uint64_t* heap_words = nullptr;
    int64_t heap_words_cap = 0;
    uint32_t heap_epoch = 0;
    // fixed: every buffer above is a view into memory the workspace does not
    // own (the allocation-free entry point's scratch array); a request beyond
    // a buffer's size fails with DM_ERR_BUDGET_EXCEEDED instead of growing it
    bool fixed = false;

    dm_status init(dm_context* c, hipStream_t s);
    void release();
    dm_status ensure_buf(int i, int64_t elems);
    dm_status ensure_status(int64_t words);
    dm_status ensure_spill(int64_t n);
    dm_status ensure_sort_scratch(int64_t elems);
    // next look-back epoch; clears status words and tickets when wrapping
    dm_status next_epoch(uint32_t* e);
    // heap of at least max(elems, min_elems) int32 and min_words look-back words
    dm_status ensure_heap(int64_t elems, int64_t min_elems, int64_t min_words);
    // epoch tagging one batched call's look-back words (clears them on wrap); 0 = error
    uint32_t next_heap_epoch();
};

// Motif table keyed on one position (see TableDev).
struct MotifTable {
    int32_t* cols[kMaxMotif] = {};  // column of each motif position (cols[p] = cols[0] + p * stride)
    int64_t stride = 0;
    int32_t* offs = nullptr;        // n_vertices + 1
    int64_t rows = 0;
    int32_t size = 0;
    // A second copy of the rows (same offsets) whose key groups are ordered
    // by position sorted_by - 1, for steps whose first further key sits there
    int32_t* sec_base = nullptr;
    bool sec_rowmajor = false;  // the second copy is row-major (size int32 per row)
    int32_t sorted_by = 0;
    int32_t sorted_max = 0;  // largest key group the second copy orders
    // run index of the row-major second copy (see TableDev::pair_offs)
    int32_t* run_offs = nullptr;
    int32_t* run_far = nullptr;
    int32_t* run_start = nullptr;
    // allocations to free (data, offs, second copy, run index)
    int32_t* owned[4] = {nullptr, nullptr, nullptr, nullptr};
};

struct DataGraph;

}  // namespace dm

namespace dm {
// Device blocks freed on the context's own stream, kept for the next
// allocation of the same size class: on that stream stream order makes the
// reuse safe; another stream (a server's worker) first waits for an event
// recorded on the context stream at that point.  A result and its release
// then cost no memory-pool round trip.  Blocks of up to kMaxBlock bytes,
// kMaxCached bytes in all.
struct BlockCache {
    static constexpr size_t kMaxBlock = (size_t)256 << 20;
    static constexpr size_t kMaxCached = (size_t)1 << 30;
    std::mutex mu;
    hipEvent_t ev = nullptr;  // recorded on the context stream before a block moves to another stream
    std::unordered_map<size_t, std::vector<void*>> bins;  // size class -> free blocks
    std::unordered_map<void*, size_t> live;               // blocks handed out from a class
    size_t cached = 0;
    // the class of a request: 4 KiB, else rounded up to a quarter of its power of two
    static size_t size_class(size_t bytes) {
        if (bytes <= 4096) return 4096;
        size_t p = 1;
        while ((p << 1) <= bytes) p <<= 1;
        const size_t step = p >> 2;
        return (bytes + step - 1) / step * step;
    }
};
}  // namespace dm

struct dm_context {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool has_alloc = false;   // the caller's allocator (else the default pool)
    dm_allocator alloc{};
    uint32_t* cancel = nullptr;  // host-coherent word polled by waiting kernels (dm_context_cancel)
    int64_t wall_khz = 100000;   // device wall-clock rate (bounded waits)
    dm::Workspace ws;
    int32_t sort_lds_max = 0;
    dm::PlanCache plans;  // by (pattern, motif set, table statistics)
    mutable dm::BlockCache blocks;  // default-pool blocks freed on `stream`
};

struct dm_datagraph {
    dm_context* ctx = nullptr;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t max_degree = 0;
    int32_t* row_ptr = nullptr;
    int32_t* col = nullptr;
    int32_t* src = nullptr;
    uint32_t* bitmap = nullptr;
    int32_t words_per_row = 0;
    uint32_t* vcost = nullptr;  // layout costs: per vertex (n) and per CSR entry (nnz); zeros until set
    uint32_t* ecost = nullptr;
    uint32_t mask_built = 0;  // DM_MOTIF_* bits
    uint32_t motif_bits = 1;  // bit per MotifIndex present
    dm::MotifTable tab[dm::kNumMotifs][6];
    dm::MotifStats stats;
    double build_ms = 0;
    std::vector<int32_t> host_row_ptr;  // CSR offsets read back at ingest (the degree sequence)
    std::atomic<int32_t> servers{0};    // servers started on this graph and not yet stopped
    // batched form's launch shape chosen by dm_autotune_batch (0 = the defaults)
    int32_t batch_block = 0, batch_grid = 0, batch_backoff = 0, batch_max_cols = 0;

    dm::GraphDev graph_dev() const {
        dm::GraphDev g;
        g.row_ptr = row_ptr;
        g.col = col;
        g.bitmap = bitmap;
        g.n = n;
        g.words_per_row = words_per_row;
        return g;
    }
    dm::TableDev table_dev(int motif, int key_pos) const;
    // the table a join step reads: the second copy when it is ordered by the
    // step's first further key
    dm::TableDev table_dev_step(const dm::StepDesc& st) const;
};

struct dm_result {
    dm_context* ctx = nullptr;
    int32_t width = 0;
    int64_t rows = 0;
    int64_t total = 0;
    int32_t* data = nullptr;  // device, row-major
    uint64_t* costs = nullptr;  // scored results: device, one per row (owned)
    std::shared_ptr<void> block;  // batched results share one allocation (data points inside)
    hipStream_t stream = nullptr;
    int32_t mode = DM_OUT_TABLE;
    uint64_t hsum = 0, hxor = 0;
    dm_run_stats stats{};
};

namespace dm {

struct RunOptions {
    int32_t block = 0;         // 0 = auto
    int32_t mode = DM_OUT_TABLE;
    bool sync_each_step = false;
    int64_t mem_budget = 0;
    int64_t cap = -1;          // max embeddings (< 0 = all)
    bool sort = true;          // canonicalize (false: keep plan-order SoA, for motif tables)
    bool profile = false;      // time each launch with events
    int64_t initial_rows = 0;  // first-attempt table capacity (0 = estimate)
    int32_t root_begin = 0;    // root range [root_begin, root_end) of the identity table;
    int32_t root_end = 0;      // empty range = every data vertex
    bool induced = false;      // pattern non-edges must map to data non-edges
    bool score = false;        // layout costs per row; with cap >= 0 the cap best rows by (cost, row)
    int64_t result_limit = 0;  // bytes the kept rows may take (0 = what device memory holds)
    int64_t wait_limit_us = 0; // bound of device waits in microseconds (0 = the default)
    // caller-owned destination of the sorted rows (row-major, out_buf_rows
    // rows); nullptr = the run allocates its result
    int32_t* out_buf = nullptr;
    int64_t out_buf_rows = 0;
};

// Bounded-wait control of one run: the run's abort word and record, the
// context's cancel word and the limit in wall-clock ticks.
WaitCtl wait_ctl(const dm_context* ctx, uint32_t* abort, WaitDiag* diag, int64_t limit_us);
// DM_OK when the run's abort word (host copy) is clear, else the failure it
// records: DM_ERR_CANCELLED, or DM_ERR_DEVICE naming the wait that gave up.
dm_status check_abort(uint32_t abort, const WaitDiag& d, const char* where);

// Output of one plan execution on one workspace.
struct RunOutput {
    int64_t rows = 0;          // final table rows (before cap)
    int32_t* table = nullptr;  // SoA final table (plan column order) when !sort, owned by workspace
    int64_t stride = 0;
    int32_t* sorted = nullptr; // row-major sorted table (ownership passes to the caller)
    int64_t sorted_rows = 0;
    uint64_t* costs = nullptr; // scored runs: cost of each sorted row (ownership passes to the caller)
    uint64_t hsum = 0, hxor = 0;
    dm_run_stats stats{};
};

dm_status run_plan(dm_context* ctx, Workspace& ws, const dm_datagraph* dg, const Plan& plan,
                   const RunOptions& opt, RunOutput* out);
// run_plan over root ranges: splits a range whose tables exceed the memory
// budget, serves a cap from the lowest ranges first; out.rows = -1 when a
// cap stopped before every range was counted.
dm_status run_plan_chunked(dm_context* ctx, Workspace& ws, const dm_datagraph* dg, const Plan& plan,
                           const RunOptions& opt, RunOutput* out);

// Canonicalize n_jobs final tables (jobs already in device memory) on
// ws.stream: two LDS tiers, then chunk sort + merge passes for the rest.
// max_in_cap / max_wp bound every job's rows and packed-row words (they size
// the number of merge passes); counters = 4 zeroed int32 in device memory
// (spill_n[2], max_chunks, dup), dup is nonzero afterwards if two rows of a
// segment were equal.
// abort: the run's abort word (the tiers do nothing once it is set).
// max_in_cap bounds every job's rows; when it exceeds the tier-2 tile the
// count of segments tier 2 passed on is read back through host_word (host
// memory) and the merge tier is launched only if there are any.  prof
// (optional, 3 events): recorded after the LDS tiers and around the merge
// tier; *merged tells whether it ran.  one (optional): a single job passed
// with the launches instead of jobs_d (n_jobs 1, merge_later required: the
// caller uploads the job before it runs the merge tier).
dm_status enqueue_sort(dm_context* ctx, Workspace& ws, const SortJob* jobs_d, int32_t n_jobs, int32_t nv,
                       int32_t v0, int64_t max_in_cap, int32_t max_wp, int32_t* counters, const uint32_t* abort,
                       int32_t* host_word, hipEvent_t* prof = nullptr, bool* merged = nullptr, int32_t stream_k = 0,
                       bool* merge_later = nullptr, const SortJob* one = nullptr);
// The merge tier over the segments tier 2 passed on (counters[1] of them,
// nonzero), for a caller that took enqueue_sort's merge_later.
dm_status enqueue_sort_merge(dm_context* ctx, Workspace& ws, const SortJob* jobs_d, int32_t n_jobs, int32_t nv,
                             int32_t v0, int64_t max_in_cap, int32_t max_wp, int32_t* counters, const uint32_t* abort,
                             hipEvent_t* prof);

dm_status plan_for(const dm_datagraph* dg, const NormPattern& p, const dm_plan_opts* opts, Plan* plan);
// zero layout costs for a data graph that has none set yet
dm_status ensure_costs(dm_datagraph* dg);
RunOptions run_options(const dm_plan_opts* opts, int64_t cap);
dm_result* empty_result(dm_context* ctx, int32_t k, int32_t mode);
// One pattern through Algorithm 1 on workspace `ws` (its stream).
dm_status enumerate_one(dm_datagraph* dg, Workspace& ws, const dm_graph_desc* gp, int64_t cap,
                        const dm_plan_opts* opts, dm_result** out);

}  // namespace dm
