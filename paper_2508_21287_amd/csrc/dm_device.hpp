// Device-side argument blocks and the host-callable kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "dm_common.hpp"

namespace dm {

// A motif table Res(M) keyed on one motif position: one SoA block, column p
// (motif position p) at base + p * stride, rows grouped by the key column in
// ascending key order, and offs[v]..offs[v+1] = the rows whose key is v
// (direct-address index).
struct TableDev {
    const int32_t* base;
    int64_t stride;   // column stride (position p of row m at base + p * stride + m * rstride)
    int64_t rstride;  // row stride: 1 for a column-major (SoA) table, `size` for a row-major one
    const int32_t* offs;
    int64_t rows;
    int32_t size;
    // 1 + the motif position by which the rows of every key group of at most
    // sorted_max rows are ascending (0: no such order)
    int32_t sorted_by;
    int32_t sorted_max;
    int32_t pad_;
    // Run index of a table ordered by (key, position sorted_by - 1): for key
    // v, the distinct values of that position are pair_far[pair_offs[v] ..
    // pair_offs[v+1]) (ascending) and the run of value pair_far[i] starts at
    // row pair_start[i] and ends where the next one starts (or at the group's
    // end).  nullptr: none.
    const int32_t* pair_offs;
    const int32_t* pair_far;
    const int32_t* pair_start;
};

constexpr int kGroupSortMax = 64;    // groups the per-thread insertion sort orders
constexpr int kGroupSortLds = 4096;  // groups the per-workgroup LDS sort orders

// Normalized data graph: CSR (each list ascending) + optional adjacency bitmap
// (bit v of row u set iff {u, v} is an edge; words_per_row 32-bit words/row).
struct GraphDev {
    const int32_t* row_ptr;
    const int32_t* col;
    const uint32_t* bitmap;
    int32_t n;
    int32_t words_per_row;
};

// Bounded waits.  Every spin of a kernel (a look-back on a predecessor
// tile, the persistent scheduler waiting for work) gives up when the device
// wall clock has advanced `limit` ticks without progress, or at once when the
// context's cancel word (host memory, set by dm_context_cancel) or the run's
// abort word is set.  The first wait to give up records what it waited for in
// `diag` and sets `abort`; every workgroup then leaves its loop normally and
// the kernels still to come in the run return at entry, so the host sees the
// record after its next readback instead of a device that never finishes.
enum { WAIT_NONE = 0, WAIT_LOOKBACK = 1, WAIT_IDLE = 2, WAIT_CANCEL = 3 };

struct WaitDiag {
    int32_t reason;     // WAIT_*
    int32_t pattern;    // batch item of the wait (-1: a single-pattern run)
    int32_t step;       // join step (idle waits: the stage of the first unfinished pattern)
    int32_t ntiles;     // tiles of that step
    int64_t tile;       // tile that waited (look-back) or -1
    int64_t spins;      // polls before giving up
    int64_t ticks;      // wall-clock ticks waited
    int32_t claimed;    // idle waits: tiles of that step claimed / finished so far
    int32_t finished;
};

struct WaitCtl {
    uint32_t* abort;         // run's abort word (device, zeroed by the host before the run)
    WaitDiag* diag;          // written once, by the wait that set `abort`
    const uint32_t* cancel;  // context's cancel word (host-coherent memory; nullptr = none)
    uint64_t limit;          // wall-clock ticks a wait may last without progress
};

enum { EJF_WRITE = 0, EJF_HASH = 1 };

// One join-filter launch.  Input table: `in` SoA with column stride
// in_stride and at most in_cap rows, row count *n_in (clamped to in_cap);
// in == nullptr means the identity table (one column, values id_begin +
// row, id_count rows).  Output: SoA with stride out_stride, at most out_cap
// rows written; *n_out receives the exact count even past out_cap, and
// *overflow is set when out_cap was too small.  Output rows keep the order of
// their input rows (order-preserving compaction via decoupled look-back over
// tiles claimed in ticket order).
struct EjfArgs {
    StepDesc st;
    TableDev tbl;
    GraphDev g;
    const int32_t* in;
    int64_t in_stride;
    int64_t in_cap;
    const int64_t* n_in;
    const int64_t* in_row0;  // device: rows of `in` start here (nullptr = 0): a motif table read in place
    int32_t id_begin;
    int32_t id_count;
    int32_t* out;
    int64_t out_stride;
    int64_t out_cap;
    int64_t* n_out;
    int32_t* overflow;
    uint64_t* status;     // look-back words, >= tiles of this launch
    uint64_t* ticket;     // tile counter, zero before the launch
    uint32_t epoch;       // tags this launch's look-back words
    int32_t mode;         // EJF_WRITE or EJF_HASH
    uint64_t* hash_acc;   // EJF_HASH: [count, sum, xor]
    // Batched form: while this step writes, *next_cand accumulates the
    // candidate count of every output row for the next step (its motif
    // index range at column next_key_col, or 1 when next_key_col < 0: a
    // filter step), an exact upper bound of the next step's output rows.
    int64_t* next_cand;   // nullptr = not needed
    const int32_t* next_offs;
    int32_t next_key_col;
    int32_t induced;      // 1: pattern non-edges must map to data non-edges (StepDesc::padj)
    int32_t cand_par;     // per-launch form: 1 = candidate-parallel tiles (many candidates per row, uneven)
    int32_t pad_cp_;
    // Layout scoring: when out_cost is set, each output row's cost is its
    // input row's cost (identity input: the root's vertex cost) plus the
    // vertex costs of the new values and the edge costs of the pattern edges
    // the new columns close (StepDesc::padj); ecost is aligned with the CSR.
    const uint32_t* vcost;
    const uint32_t* ecost;
    const uint64_t* in_cost;
    uint64_t* out_cost;
    WaitCtl w;            // bounded look-back (see WaitCtl)
    int32_t diag_pattern; // batch item and step named by a wait that gives up
    int32_t diag_step;
    uint8_t pv[kMaxCols]; // EJF_HASH: pattern vertex of each output column
};

// Canonicalization of one final table: permute columns to pattern-vertex
// order, sort the rows of each root segment (rows sharing column 0)
// lexicographically, write rows [0, out_rows) of the sorted table row-major.
struct SortJob {
    const int32_t* in;
    int64_t in_stride;
    int64_t in_cap;
    const int64_t* n_in;
    const int64_t* in_row0;  // device: rows of `in` start here (nullptr = 0): a motif table read in place
    int32_t* out;
    int64_t out_rows;
    uint32_t* scratch_idx;  // merge tier: 2 * in_cap index scratch
    const uint64_t* in_cost;  // per input row cost (nullptr = none); permuted with the rows into out_cost
    uint64_t* out_cost;
    int32_t k;
    // LDS rows are packed: columns 1..k-1 (pattern order) at `bits` bits
    // each, cpw per 64-bit word, the earlier column in the higher bits, so
    // comparing the words in order compares the rows lexicographically
    int32_t wp;             // words per packed row (odd)
    int32_t bits;
    int32_t cpw;
    int32_t pad_;
    uint8_t perm[kMaxCols]; // pattern vertex j -> input column
};

// Packed-row layout for k columns of vertex ids below n_vertices.
inline void sort_pack_layout(int k, int32_t n_vertices, SortJob* j) {
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n_vertices) bits++;
    j->bits = bits;
    j->cpw = 64 / bits;
    const int w = k > 1 ? (k - 1 + j->cpw - 1) / j->cpw : 1;
    j->wp = w | 1;
}

// A root segment passed from one sort tier to the next: rows
// [seg0, seg0 + len) of job item / n_vertices.
struct SegRef {
    int32_t item;
    int32_t pad_;
    int64_t seg0;
    int64_t len;
};

// One sort launch over n_jobs tables; item = job * n_vertices + (v - v_begin)
// for every root vertex v (list == nullptr), or the segments in `list`.
// Segments that do not fit this tier's LDS are appended to `spill`.
struct SortLaunch {
    const SortJob* jobs;
    int32_t n_jobs;
    int32_t n_vertices;
    int32_t v_begin;
    int32_t lds_bytes;
    const SegRef* list;
    const int32_t* list_n;
    SegRef* spill;
    int32_t* spill_n;
    int32_t* dup_count;
    int32_t* max_chunks;  // merge tier: most LDS chunks of any listed segment
    int32_t pass;         // merge tier: pass number of a merge launch
    const uint32_t* abort;// nonzero: a wait of the run gave up; the launch does nothing
    const uint32_t* todo; // LDS tiers without a list: only items whose word equals todo_epoch (nullptr = all)
    uint32_t todo_epoch;  // the streaming pass sets the words of the segments it finds out of order to this
    int32_t pad_;
    SortJob one;          // the job when `jobs` is nullptr (one table, passed with the launch)
};

// Packed rows of wp 64-bit words that an LDS tile of lds_bytes holds
// together with the 16-bit index array of the bitonic network (padded to a
// power of two P): the best r <= P over P with 8 * wp * r + 2 * P <= lds_bytes.
__host__ __device__ inline int lds_rows_of(int lds_bytes, int wp) {
    int best = 0;
    for (int P = 1; P <= 65536 && 2 * P < lds_bytes; P <<= 1) {
        int r = (lds_bytes - 2 * P) / (8 * wp);
        if (r > P) r = P;
        if (r > 65535) r = 65535;  // 0xFFFF is the index sentinel
        if (r > best) best = r;
    }
    return best;
}

// Batched form: per-pattern progress of the persistent join kernel.
struct BatchCtl {
    int32_t stage;  // step being processed; == n_steps once retired
    int32_t pad_[3];
    int64_t cand[kMaxSteps];  // upper bound of step s's output rows (see EjfArgs::next_cand)
    int32_t ntiles[kMaxSteps];
    int32_t claim[kMaxSteps];
    int32_t done[kMaxSteps];
    int64_t n_in[kMaxSteps];
    int64_t t_pub[kMaxSteps + 1];  // device wall clock when step s was published (s = n_steps: retired)
};

// Device heap of the batched form: when a step is published, its output
// table (rows = the exact candidate bound) and its look-back words are cut
// from these arrays by bump allocation; a pattern whose tables do not fit
// is retired with heap_fail set and redone by the host.
struct BatchDev {
    EjfArgs* args;         // all (pattern, step) argument blocks; out/in/status filled on publication
    const int32_t* first;  // per pattern: index of its step 0 in args
    const int32_t* nsteps; // per pattern
    BatchCtl* ctl;         // per pattern, zeroed except ntiles[0]/n_in[0]
    int32_t* finished;     // retired patterns
    int32_t* heap_fail;    // per pattern: 1 = its tables did not fit the heap
    SortJob* jobs;         // per pattern: in/in_stride/in_cap/scratch_idx set when its last step ends
    int32_t* heap;
    int64_t heap_cap;      // int32 elements
    unsigned long long* heap_top;
    uint64_t* words;
    int64_t words_cap;
    unsigned long long* words_top;
    int64_t row_limit;     // > 0: cap every step's output capacity (forces the overflow path)
    int32_t n_patterns;
    int32_t max_backoff;   // idle polling backoff cap (units of s_sleep(16))
    WaitCtl w;             // bounded idle waits (progress = tiles_done advancing)
    uint32_t* tiles_done;  // tiles finished by every workgroup so far
};

// Top-k by (cost, table position): radix selection of the k-th key, then a
// gather and a sort of the k winners.
struct TopkCtl {
    unsigned long long prefix;  // selected high bits of the threshold cost / position
    long long k_rem;            // rank still to place inside the current prefix class (1-based)
    long long n_less;           // rows with cost below the threshold
    unsigned long long n_out;   // gathered winners
    unsigned int hist[256];
    unsigned long long t_cost;  // threshold cost after the cost passes
};
constexpr int kTopkMax = 8192;  // winners sorted in one workgroup's LDS

constexpr int kEpochBits = 14;
constexpr uint32_t kEpochs = 1u << kEpochBits;

// ---- launchers (kernels.hip) ----
// block size the join launch uses for c_in input columns (requested 0 = auto);
// wide rows take smaller tiles so the LDS row tile stays small
int ejf_block_for(int c_in, int requested);
hipError_t launch_ejf(const EjfArgs& a, int block, int grid, hipStream_t s);
// threads: workgroup size, a multiple of 64 up to 1024
hipError_t launch_sort_lds(const SortLaunch& a, int grid, int threads, int lds_bytes, hipStream_t s);
// One job's table (n_jobs == 1) in one streaming pass: every kept row written
// to its place in the output (row-major, pattern order), the bit of each root
// segment that is out of order set in `unsorted` (one bit per item, counted
// in *n_unsorted), and duplicate neighbours counted.  The LDS tiers then sort
// only the flagged segments.  in_cap_rows bounds the grid.
hipError_t launch_sort_stream(const SortLaunch& a, uint32_t* unsorted, int32_t* n_unsorted, int64_t in_cap_rows, int k,
                              hipStream_t s);
// chunk sort + `passes` merge launches + row write for the segments in a.list
hipError_t launch_sort_merge_tier(const SortLaunch& a, int passes, hipStream_t s);
// The k (<= kTopkMax, <= n) rows of `table` (row-major, n x width) with the
// smallest (cost, position) keys, in that order: rows to out_rows, costs to
// out_cost.  ctl and the k-entry scratch (sel_cost, sel_pos) are device memory.
hipError_t launch_topk(const uint64_t* cost, int64_t n, int64_t k, TopkCtl* ctl, uint64_t* sel_cost,
                       uint32_t* sel_pos, const int32_t* table, int32_t width, int32_t* out_rows,
                       uint64_t* out_cost, hipStream_t s);
// Batched form: workgroup size (= tile rows) for inputs up to max_cols
// columns (requested 0 = auto), the grid (requested 0 = 1024, at most what
// stays resident) and the launch; max_cols sizes the LDS row tile.
int batch_block_for(int max_cols, int requested);
int batch_grid_for(int block, int max_cols, int requested);
// wide: some step adds more than kNarrowNew values (the wide instantiation)
hipError_t launch_batch(const BatchDev& b, int block, int max_cols, bool wide, int grid, hipStream_t s);
int sort_max_lds_bytes();
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
// *row0 = offs[v0], *n = offs[v1] - offs[v0]: the rows of keys [v0, v1) of a motif table
hipError_t launch_slice_rows(const int32_t* offs, int32_t v0, int32_t v1, int64_t* n, int64_t* row0, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// p[0..n) = 0 except p[at] = v
hipError_t launch_clear_set_u64(uint64_t* p, int64_t n, int64_t at, uint64_t v, hipStream_t s);
hipError_t launch_iota_i32(int32_t* p, int32_t start, int64_t n, hipStream_t s);
hipError_t launch_offsets(const int32_t* key, const int64_t* n_rows, int64_t rows_cap, int32_t n_vertices,
                          int32_t* offs, hipStream_t s);
hipError_t launch_gather_cols(const int32_t* in, int64_t in_stride, const int64_t* n_rows, int64_t cap,
                              const int32_t* colmap, int32_t ncols, int32_t* out, int64_t out_stride,
                              hipStream_t s);

// graph ingest
hipError_t launch_ingest_count(const int32_t* edges, int64_t m, int32_t n, int32_t* deg, int32_t* err,
                               hipStream_t s);
// look-back words tagged with `epoch` (words of other epochs read as not
// ready, so nothing is cleared first); the tile ticket is tickets[epoch]
hipError_t launch_scan_i32(const int32_t* in, int32_t* out_excl, int64_t n, int64_t* total,
                           uint64_t* status, uint64_t* tickets, uint32_t epoch, const WaitCtl& w, hipStream_t s);
// up to kHostGather device ranges (sizes in bytes, multiples of 4, 4-byte
// aligned) into pinned host memory, one launch
constexpr int kHostGather = 6;
struct HostGather {
    const void* src[kHostGather];
    void* dst[kHostGather];
    int64_t bytes[kHostGather];
    int32_t n;
    int32_t pad_;
};
hipError_t launch_gather_to_host(const HostGather& g, hipStream_t s);
// edges with an endpoint outside [0, n) are skipped (ingest_count flags them)
hipError_t launch_ingest_scatter(const int32_t* edges, int64_t m, int32_t n, const int32_t* ptr, int32_t* cursor,
                                 int32_t* tmp, hipStream_t s);
hipError_t launch_ingest_sort_small(const int32_t* ptr, int32_t* tmp, int32_t n, int32_t* udeg,
                                    int32_t* big, int32_t* big_n, hipStream_t s);
hipError_t launch_ingest_sort_big(const int32_t* ptr, int32_t* tmp, int32_t* udeg, const int32_t* big,
                                  const int32_t* big_n, int32_t* err, hipStream_t s);
hipError_t launch_ingest_compact(const int32_t* tmp_ptr, const int32_t* tmp, const int32_t* row_ptr,
                                 int32_t n, int32_t* col, int32_t* src, int32_t* max_deg, hipStream_t s);
// The claw table (centre 0, leaves 1..3) from the CSR: per key vertex row
// counts (key_pos 0: centre, 1: leaf), then the rows at the scanned offsets
// (SoA, column stride `stride`)
hipError_t launch_claw_count(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos, int32_t* cnt,
                             hipStream_t s);
hipError_t launch_claw_fill(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos, const int32_t* offs,
                            int64_t stride, int32_t* data, hipStream_t s);
// Sort the rows of every key group of at most kGroupSortMax rows (group v =
// rows [offs[v], offs[v+1]) of the SoA table data, `size` <= 6 columns of
// stride `stride`) by column `sec`, stably
hipError_t launch_group_sort(const int32_t* offs, int32_t n, int64_t stride, int32_t size, int32_t sec, int32_t* data,
                             hipStream_t s);
// The same order for groups of up to cap rows (a power of two, at most
// kGroupSortLds), any number of columns, from the SoA table `in` into `out`,
// row-major (size int32 per row; larger groups copied in their order)
hipError_t launch_group_sort_lds(const int32_t* offs, int32_t n, int64_t stride, int32_t size, int32_t sec,
                                 const int32_t* in, int32_t* out, int32_t cap, hipStream_t s);
// Run index of a row-major table of `rows` rows (`size` int32 each) ordered
// by (column 0, column sec): flags[i] = 1 where a run starts (the scan of the
// flags gives each run its index), then the runs' first rows and values, and
// each key's first run (see TableDev::pair_offs)
hipError_t launch_run_flags(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, int32_t* flags,
                            hipStream_t s);
hipError_t launch_run_fill(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, const int32_t* flags,
                           const int32_t* idx, int32_t* run_far, int32_t* run_start, hipStream_t s);
hipError_t launch_run_offs(const int32_t* offs, int32_t n, int64_t rows, const int32_t* idx, const int64_t* total,
                           int32_t* run_offs, hipStream_t s);
// flags[0] |= 1: the graph (ascending merged CSR lists) has a 4-cycle;
// flags[1] |= 1: a vertex of degree above 16 left the answer undecided
hipError_t launch_c4_check(const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t* flags, hipStream_t s);
// *nnz_dev (<= nnz_max) directed edges, read on the device
hipError_t launch_bitmap_set(const int32_t* src, const int32_t* col, const int64_t* nnz_dev, int64_t nnz_max,
                             int32_t wpr, uint32_t* bitmap, hipStream_t s);

}  // namespace dm
