/*
 * dmotif.h -- C ABI of libdmotif.so: subgraph-embedding enumeration as
 * relational operations on int32 tables (the Delta-Motif method), on AMD
 * Instinct MI355X (gfx950) with hand-written HIP kernels.
 *
 * The two central calls mirror the paper's two procedures:
 *   dm_datagraph_build  -- Algorithm 2 (BuildDatabase): normalize the data
 *                          graph and build its motif tables Res(M) once,
 *                          resident in device memory.
 *   dm_enumerate        -- Algorithm 1 (the join-and-filter loop): decompose
 *                          the pattern into motif slices (Sec. III-C), join
 *                          partial-embedding tables with the motif tables on
 *                          shared pattern-vertex columns (Sec. III-B), filter
 *                          for injectivity and pattern-edge consistency, then
 *                          sort into the canonical embedding table.
 * The problem is the one stated in Sec. III-A: every injective map
 * f : V_p -> V_d that sends each pattern edge to a data edge ("non-induced"
 * reading: the join and the filter enforce edge preservation and
 * injectivity; extra data edges between images are allowed).
 *
 * Conventions shared by every call:
 *  - Every function returns dm_status; outputs are written only on DM_OK.
 *    dm_last_error() gives a thread-local message for the last failure.
 *  - Graph inputs are HOST arrays of undirected (u, v) int32 pairs, row-major
 *    [n_edges][2].  The library copies them; the caller keeps ownership.
 *  - Data graph: ids must lie in [0, n_vertices) (else DM_ERR_VERTEX_RANGE);
 *    self-loops are dropped and repeated edges merged (Sec. III-D: Res(M2)
 *    is E_d without self-loops, both orientations present).
 *  - Pattern: ids in [0, n_vertices) (else DM_ERR_VERTEX_RANGE), no self-loop
 *    (DM_ERR_PATTERN_SELF_LOOP), connected (DM_ERR_PATTERN_DISCONNECTED);
 *    repeated edges merge.  1 <= n_vertices <= DM_MAX_PATTERN_VERTICES.
 *    A 1-vertex pattern yields every data vertex; a pattern with more
 *    vertices than the data graph yields 0 rows (DM_OK).
 *  - Results: row-major int32 [rows][width], width = pattern vertex count,
 *    column j = f(j), rows in ascending lexicographic order, no duplicates.
 *    A cap (max_embeddings >= 0) keeps the lexicographically first `cap`
 *    rows; the total count is still reported unless early exit stopped it.
 *  - Handles are owned by the library until the matching *_free/_destroy.
 *    Device pointers inside a result live until dm_result_free.
 *  - Work is stream-ordered on the context's HIP stream.  dm_enumerate
 *    returns once the row count is known on the host (one device->host
 *    sync); the device table is complete when the stream reaches that point.
 *  - Threading: a context is used by one host thread at a time (its calls
 *    share the context's workspace).  A data graph is only read by the
 *    enumeration calls, so a server's worker threads (each with a workspace
 *    and stream of its own) and the context's thread may enumerate on it at
 *    once; the calls that change or release it (dm_datagraph_set_costs,
 *    dm_datagraph_free) return DM_ERR_BUSY while a server holds it.  A
 *    server is internally synchronized; dm_context_cancel may be called from
 *    any thread.
 */
#ifndef DMOTIF_H
#define DMOTIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DM_MAX_PATTERN_VERTICES 128
#define DM_MAX_MOTIF_VERTICES 18

typedef enum {
    DM_OK = 0,
    DM_ERR_INVALID_ARG = -1,
    DM_ERR_VERTEX_RANGE = -2,
    DM_ERR_PATTERN_DISCONNECTED = -3,
    DM_ERR_PATTERN_SELF_LOOP = -4,
    DM_ERR_OUT_OF_MEMORY = -5,
    DM_ERR_BUDGET_EXCEEDED = -6,
    DM_ERR_DEVICE = -7,
    DM_ERR_CANCELLED = -8,
    DM_ERR_BUSY = -9,
    DM_ERR_TIMEOUT = -10,
    DM_ERR_INTERNAL = -11,
    DM_ERR_UNSUPPORTED = -12
} dm_status;

/* Motif families (Sec. III-A "Motifs": M_i is a path of i vertices, the
 * suffix -O a cycle).  M2 (the edge table) is always present.  A data graph
 * is built with a mask of these; a plan may use any subset of what was built.
 * DM_MOTIF_AUTO is topology-aware (Sec. VI-B): on a graph with 4-cycles
 * (grid-like) it builds M3, M4 and M4-O; without them and with low degrees
 * (heavy-hex-like: at most 5e7 claws) the claw M4-1 (as in the paper's
 * {M2, M4-1}); on either, at degrees up to 4, also M7 while its table stays
 * moderate (it covers the pattern's chains: vertices of pattern degree 2);
 * otherwise M3, M4 and, when its table stays moderate, the 12-cycle M12-O.
 * Each pattern's plan is the one with the least estimated table work among
 * the greedy decompositions with every motif built, without M7, and without
 * the paths (M3..M7). */
#define DM_MOTIF_M3 (1u << 0)
#define DM_MOTIF_M4 (1u << 1)
#define DM_MOTIF_M5 (1u << 2)
#define DM_MOTIF_M6 (1u << 3)
#define DM_MOTIF_C4 (1u << 4)
#define DM_MOTIF_C6 (1u << 5)
#define DM_MOTIF_C12 (1u << 6)
/* General shapes (Sec. VI-B): M4-1 = the claw K1,3 (centre + 3 leaves),
 * M6-2O = the 2x3 grid (two squares sharing an edge), M18-O-6 = the
 * heavy-hex cell (a 12-cycle) with a pendant vertex at every other vertex. */
#define DM_MOTIF_M4_1 (1u << 7)
#define DM_MOTIF_M6_2O (1u << 8)
#define DM_MOTIF_M18_O_6 (1u << 9)
/* M7 = the 7-vertex path, kept keyed at its ends only, each key group ordered
 * by the far end: it closes 12-cycles as one two-key join of two 7-paths
 * (Alg. 2 builds it from M4 joined with M4; Sec. III-D, larger motifs from
 * joins of smaller ones). */
#define DM_MOTIF_M7 (1u << 10)
#define DM_MOTIF_ALL 0x7FFu
#define DM_NUM_MOTIFS 12
#define DM_MOTIF_AUTO 0u
/* For dm_plan_opts.motif_mask: plan with M2 only (Sec. IV-B: one join per
 * pattern edge, the parallel analogue of tree search). */
#define DM_MOTIF_M2_ONLY 0x80000000u

typedef struct {
    int32_t n_vertices;
    int64_t n_edges;
    const int32_t* edges; /* host, [n_edges][2] */
} dm_graph_desc;

typedef enum {
    DM_OUT_TABLE = 0,      /* materialize the sorted embedding table */
    DM_OUT_COUNT_HASH = 1  /* count + order-independent multiset hash only */
} dm_output_mode;

typedef struct {
    uint32_t motif_mask;   /* motifs the planner may use; 0 = every motif built */
    int32_t block_threads; /* join-kernel workgroup size (64, 128, 256); 0 = auto */
    int32_t output_mode;   /* dm_output_mode */
    int32_t sync_each_step;/* 1: read each step's row count back (exact sizing) */
    int64_t mem_budget;    /* bytes for intermediate tables; 0 = library default (48 GiB) */
    int32_t profile;       /* 1: time every join and sort launch with HIP events (see dm_run_stats) */
    int32_t induced;       /* 1: induced embeddings (the definition of Sec. III-A read as "if and only
                              if"): additionally every pair of non-adjacent pattern vertices maps to
                              non-adjacent data vertices.  0 = non-induced (the method's join). */
    int64_t initial_rows;  /* first-attempt capacity of each intermediate table in rows; 0 = from the
                              planner's estimate.  Too small only costs a re-run with exact sizes. */
    int32_t root_begin;    /* keep only embeddings with f(0) in [root_begin, root_end); */
    int32_t root_end;      /* root_end <= root_begin = every data vertex.  Disjoint root ranges
                              partition the result (a shard of one pattern's enumeration). */
    int32_t score;         /* 1: layout scoring (Sec. VI-D): every row gets the cost
                              sum_v c(f(v)) + sum_{uv in E_p} c({f(u),f(v)}) from the costs set with
                              dm_datagraph_set_costs, accumulated join by join; with a cap k >= 0
                              the result is the k rows with the smallest (cost, row) keys in that
                              order (k <= 8192, else DM_ERR_UNSUPPORTED); with no cap, every row in
                              lexicographic order with its cost.  Table mode only (the count+hash
                              mode ignores it); batches run scored patterns one by one. */
    int32_t result_mb;     /* the most the kept rows may take, in MiB (rows x pattern vertices x 4
                              bytes); beyond it the call fails with DM_ERR_BUDGET_EXCEEDED as soon
                              as the rows produced so far pass it.  0 = no limit but device memory:
                              a result assembled from root-range parts needs its bytes twice (the
                              parts, then the one result buffer) next to mem_budget of tables. */
    int32_t wait_limit_us; /* bound, in microseconds, of every device-side wait of the run (a
                              look-back on a predecessor tile, the persistent scheduler waiting for
                              work): when the device clock advances this long with no progress the
                              wait gives up, the run's remaining launches do nothing and the call
                              fails with DM_ERR_DEVICE naming the wait (pattern, step, tile,
                              polls); the context stays usable.  0 = 10 s. */
} dm_plan_opts;

typedef struct dm_context dm_context;
typedef struct dm_datagraph dm_datagraph;
typedef struct dm_result dm_result;
typedef struct dm_server dm_server;

/* Version string of the library build. */
const char* dm_version(void);

/* Thread-local description of the most recent failure on this thread. */
const char* dm_last_error(void);

/* Device-memory allocator of a context.  alloc returns `bytes` of device
 * memory usable by work ordered on `stream` (a hipStream_t), or NULL on
 * failure; free returns a pointer alloc gave, after the work already queued
 * on `stream` (stream-ordered, like hipFreeAsync).  `user` is passed back to
 * both.  Both callbacks may be called from any thread that uses the context
 * (server worker threads included) and must be thread-safe.  Every device
 * buffer the library holds (tables, workspaces, results) comes from it;
 * pinned host staging buffers do not. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* stream, void* user);
    void* user;
} dm_allocator;

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t; NULL = a stream the context creates and owns).  `alloc`
 * (copied; may be NULL = stream-ordered allocation from the device's default
 * memory pool) supplies every device buffer of the context and of the data
 * graphs, results and servers made from it; a NULL return from alloc.alloc
 * makes the call that needed the memory fail with DM_ERR_OUT_OF_MEMORY,
 * freeing what that call had taken, and leaves the context usable.
 * Errors: DM_ERR_INVALID_ARG (bad device, out == NULL, an allocator with a
 * NULL callback -- checked before any device call), DM_ERR_DEVICE. */
dm_status dm_context_create(int32_t device, void* hip_stream, const dm_allocator* alloc, dm_context** out);
/* Free data graphs, results and servers created on a context before destroying it. */
void dm_context_destroy(dm_context* ctx);

/* Set (flag != 0) or clear the context's cancel word.  While it is set,
 * dm_enumerate and dm_enumerate_batch calls on the context (and on servers
 * of its data graphs) fail with DM_ERR_CANCELLED, and kernels of the
 * context that are waiting -- the persistent batch kernel at its start and
 * while idle, any look-back -- give up and leave normally, so a running
 * call returns DM_ERR_CANCELLED without leaving work on the device.  The word
 * stays set until cleared.  Callable from any thread (one host store into
 * host-coherent memory the kernels poll).  Errors: DM_ERR_INVALID_ARG. */
dm_status dm_context_cancel(dm_context* ctx, int32_t flag);

/* Algorithm 2 (BuildDatabase): normalize `gd` into device CSR + adjacency
 * bitmap and build the motif tables selected by `motif_mask` (DM_MOTIF_*),
 * each sorted by a key column with a direct-address (CSR-offset) index.
 * The result stays resident until dm_datagraph_free.
 * Errors: DM_ERR_INVALID_ARG, DM_ERR_VERTEX_RANGE, DM_ERR_OUT_OF_MEMORY,
 * DM_ERR_UNSUPPORTED (a vertex degree above 16384), DM_ERR_DEVICE. */
dm_status dm_datagraph_build(dm_context* ctx, const dm_graph_desc* gd, uint32_t motif_mask,
                             dm_datagraph** out);
/* Release the data graph's device memory, ordered after the work already
 * queued on the context stream (no wait).  Errors: DM_ERR_BUSY (a server
 * started on it has not been stopped; nothing is released). */
dm_status dm_datagraph_free(dm_datagraph* dg);

typedef struct {
    int32_t n_vertices;
    int64_t n_directed_edges; /* 2|E| after normalization */
    int32_t max_degree;
    int32_t has_bitmap;       /* adjacency bitmap built (|V| <= 32768) */
    uint32_t motif_mask;      /* motifs actually built */
    int64_t motif_rows[DM_NUM_MOTIFS]; /* rows of Res(M) for M2,M3,M4,M5,M6,C4,C6,C12,M4-1,M6-2O,
                                          M18-O-6,M7 (0 = absent) */
    double build_ms;          /* device time of the whole build */
} dm_datagraph_info;

dm_status dm_datagraph_query(const dm_datagraph* dg, dm_datagraph_info* out);
/* Host copies of the normalized CSR: row_ptr[n+1], col[2|E|] (each list ascending). */
dm_status dm_datagraph_copy_csr(const dm_datagraph* dg, int32_t* row_ptr, int32_t* col);
/* Host copy of a motif table: motif index 0..DM_NUM_MOTIFS-1 as in motif_rows, key
 * position `key_pos` (0 for cycles; 0..ceil(size/2)-1 for paths; 0..1 for M4-1
 * (centre, leaf) and M6-2O (corner, middle); 0..2 for M18-O-6 (cycle vertex
 * with pendant, cycle vertex without, pendant)).  Rows are
 * grouped by the key column in ascending key order; columns are in motif
 * position order.  rows and width receive the shape; dst may be NULL to query. */
dm_status dm_datagraph_copy_motif(const dm_datagraph* dg, int32_t motif, int32_t key_pos,
                                  int32_t* dst, int64_t max_rows, int64_t* rows, int32_t* width);

/* Persist the database of `dg` -- the output of Algorithm 2: the normalized
 * CSR and every built motif table with its key index -- to the file `path`,
 * so that a later process reloads it instead of rebuilding it (Sec. II-A and V-B: the
 * data preparation depends only on the device topology and is cached).
 * Host file I/O after device-to-host copies on the context stream.
 * File image (little-endian): "DMOTIFDB", u32 version (2), u32 0, i32 n,
 * i64 nnz, u32 motif mask, u32 motif bits, f64 table rows[DM_NUM_MOTIFS], f64 mean
 * degree, i32 row_ptr[n+1], i32 col[nnz]; then for every built motif except
 * M2 (which is the CSR), for every key position: i64 rows, i32 width, the
 * columns i32[width][rows] in motif position order, i32 index[n+1]; last a
 * u64 FNV-1a checksum of all preceding bytes.
 * Errors: DM_ERR_INVALID_ARG (NULL argument, file cannot be written), DM_ERR_DEVICE. */
dm_status dm_datagraph_save(const dm_datagraph* dg, const char* path);

/* Reload a database written by dm_datagraph_save onto the device of `ctx`.
 * The file is validated before anything is created (magic, version,
 * checksum, vertex ids in range, monotone indexes, table widths); the CSR's
 * source column and the adjacency bitmap are rebuilt on the device exactly
 * as dm_datagraph_build does, the motif tables are uploaded as stored.
 * Several databases (for example one per device topology) may be resident
 * on one context at once.  build_ms in dm_datagraph_info reports the load
 * time.  Errors: DM_ERR_INVALID_ARG (NULL argument, unreadable, damaged or
 * foreign file), DM_ERR_OUT_OF_MEMORY, DM_ERR_DEVICE. */
dm_status dm_datagraph_load(dm_context* ctx, const char* path, dm_datagraph** out);

/* Layout-scoring costs of the data graph (Sec. VI-D: per-qubit and
 * per-coupling quality): vertex_cost[n_vertices] (NULL = all zero) and, for
 * n_cost_edges listed data edges (cost_edges: (u,v) pairs, each edge at most
 * once, either orientation), edge_cost[n_cost_edges]; unlisted edges cost 0.
 * Costs are non-negative integers (for fidelities: fixed-point -log values),
 * summed exactly in 64 bits.  Replaces earlier costs; host arrays are copied.
 * Errors: DM_ERR_INVALID_ARG (NULL, a listed pair that is not an edge of the
 * graph or is listed twice), DM_ERR_BUSY (a server holds the graph),
 * DM_ERR_OUT_OF_MEMORY, DM_ERR_DEVICE. */
dm_status dm_datagraph_set_costs(dm_datagraph* dg, const uint32_t* vertex_cost, int64_t n_cost_edges,
                                 const int32_t* cost_edges, const uint32_t* edge_cost);

/* Motif-set tuning (Sec. VI-B: the best motif set depends on the topology):
 * for each of n_candidates DM_MOTIF_* masks (DM_MOTIF_AUTO and
 * DM_MOTIF_M2_ONLY allowed), build the data graph `gd` with that set and
 * enumerate the n_sample patterns in `sample` as one batch in count+hash
 * mode, reps times; the median wall time of build + enumeration goes to
 * ms_per_candidate[c] (may be NULL) and the fastest mask to *best_mask
 * (the first one on ties).  Synchronous on the context stream.
 * Errors: DM_ERR_INVALID_ARG, and any error of the builds or enumerations. */
dm_status dm_autotune_motifs(dm_context* ctx, const dm_graph_desc* gd, int32_t n_sample,
                             const dm_graph_desc* sample, const uint32_t* candidates, int32_t n_candidates,
                             int32_t reps, uint32_t* best_mask, double* ms_per_candidate);

/* Launch shape of the batched form's persistent join launch. */
typedef struct {
    int32_t block_threads;   /* workgroup size: 64, 128 or 256 */
    int32_t grid;            /* workgroups of the launch */
    int32_t backoff;         /* most s_sleep pauses between two polls of an idle scheduler wave */
    int32_t reserved;
    double ms;               /* median time of one batched call on the sample */
} dm_batch_tuning;

/* Autotuner of the batched form (Sec. IV-C: parallelism across join-filter
 * operations): times dm_enumerate_batch on `sample` (count+hash mode, `reps`
 * calls per candidate) for each launch shape that fits the sample's widest
 * step: block sizes of 256/128/64 threads as the row width allows, grids of
 * 0.75x to 1.5x one 256-thread workgroup per CU (capped at what can be
 * resident), idle-poll backoffs of 7, 15 and 31 pauses.  The fastest shape is kept on the data graph and used by its
 * later batched calls (and server batches) whose widest step it fits; other
 * calls keep the defaults.  *best receives it; tried (may be NULL) receives
 * up to tried_cap candidates with their medians, *n_tried how many were run.
 * Synchronous on the context stream.  Errors: DM_ERR_INVALID_ARG, and any
 * error of the batched calls (the data graph then keeps its previous shape). */
dm_status dm_autotune_batch(dm_datagraph* dg, int32_t n_sample, const dm_graph_desc* sample, int32_t reps,
                            dm_batch_tuning* best, dm_batch_tuning* tried, int32_t tried_cap, int32_t* n_tried);

/* Planner only (host, no device work): decompose a pattern with the motifs
 * in `motif_mask` (Sec. III-C) and serialize the plan into `buf` as int32:
 *   [k, n_steps, col_of[k] (pattern vertex -> table column), then per step:
 *    motif (0..DM_NUM_MOTIFS-1, -1 = filter only), key_pos, key_col, c_in,
 *    n_new, new_pos[n_new], n_eq, (col, pos)[n_eq], n_edge, (col_a, col_b)[n_edge],
 *    slice_len, slice[slice_len] (pattern vertices in motif order)].
 * *len receives the number of int32 written (or needed, if buf is too small:
 * then DM_ERR_INVALID_ARG).  Errors as for pattern validation. */
dm_status dm_plan(const dm_graph_desc* gp, uint32_t motif_mask, int32_t* buf, int32_t buf_cap,
                  int32_t* len);

/* Predicted table sizes for `gp` on `dg` (host estimate from motif-table
 * sizes): est_rows = predicted embeddings, peak_bytes = predicted peak of
 * two consecutive intermediate tables. */
dm_status dm_estimate(dm_datagraph* dg, const dm_graph_desc* gp, const dm_plan_opts* opts,
                      int64_t* peak_bytes, int64_t* est_rows);

/* Algorithm 1: all embeddings of `gp` in the data graph.  max_embeddings < 0
 * = all; otherwise the lexicographically first max_embeddings rows.  opts may
 * be NULL (defaults).  Errors: pattern validation codes, DM_ERR_OUT_OF_MEMORY,
 * DM_ERR_BUDGET_EXCEEDED (one root vertex alone exceeds mem_budget, or the kept
 * rows exceed result_mb, or with result_mb = 0 what device memory can hold),
 * DM_ERR_DEVICE, DM_ERR_INTERNAL (a duplicate row reached the output). */
dm_status dm_enumerate(dm_datagraph* dg, const dm_graph_desc* gp, int64_t max_embeddings,
                       const dm_plan_opts* opts, dm_result** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * enumeration as dm_enumerate, with no device allocation of any kind.  Every
 * intermediate buffer of the run (the join tables, look-back words, tickets,
 * control block and the sort's lists and index scratch) lives in one fixed
 * device array of DM_NOALLOC_SCRATCH_MB MiB compiled into the library; each
 * device the library runs on holds its own copy until the process ends.
 *
 * out: caller-owned device buffer of out_rows_cap rows of |V_p| int32,
 *   receiving the lexicographically sorted rows (the first max_embeddings
 *   when max_embeddings >= 0), row-major.  NULL or out_rows_cap == 0 in
 *   table mode: only the count is produced (no sort).  Unused in count+hash
 *   mode (opts->output_mode).
 * rows: rows written; total: all embeddings; hash_sum / hash_xor (may be
 *   NULL): the count+hash mode's multiset hash (see dm_result_hash).
 * opts: as dm_enumerate; mem_budget, result_mb are ignored (the scratch
 *   bounds the tables); score and profile are DM_ERR_UNSUPPORTED.
 * Returns after the device work has finished (one readback).
 * Errors: pattern validation codes; DM_ERR_BUDGET_EXCEEDED when an
 *   intermediate table does not fit the scratch (the data graph, rows x
 *   columns of the widest table and the sort's index scratch share it), or
 *   when the kept rows exceed out_rows_cap (then *total holds the count and
 *   out holds the first out_rows_cap rows); DM_ERR_DEVICE, DM_ERR_CANCELLED.
 * Calls on one device share its array: the library runs them one at a time
 * (a per-device lock held for the whole call), and a call leaves the array
 * holding its own tables, which the next call overwrites. */
#define DM_NOALLOC_SCRATCH_MB 64
dm_status dm_enumerate_noalloc(dm_datagraph* dg, const dm_graph_desc* gp, int64_t max_embeddings,
                               const dm_plan_opts* opts, int32_t* out, int64_t out_rows_cap, int64_t* rows,
                               int64_t* total, uint64_t* hash_sum, uint64_t* hash_xor);

/* Batched Algorithm 1: `n` patterns against the same resident data graph in
 * one persistent-kernel launch (per-pattern plans, device work queue).
 * caps may be NULL (all).  outs[i] receives pattern i's result; on error no
 * result is returned.  Same row semantics as dm_enumerate. */
dm_status dm_enumerate_batch(dm_datagraph* dg, int32_t n, const dm_graph_desc* gps,
                             const int64_t* caps, const dm_plan_opts* opts, dm_result** outs);

int64_t dm_result_rows(const dm_result* r);   /* rows held = min(cap, total) */
int64_t dm_result_total(const dm_result* r);  /* all embeddings; -1 if a cap stopped counting */
int32_t dm_result_width(const dm_result* r);  /* |V_p| */
/* Device pointer to the row-major table (NULL when rows == 0 or in
 * count+hash mode).  Owned by the result. */
const int32_t* dm_result_device_data(const dm_result* r);
/* Count+hash mode summaries: sum (mod 2^64) and XOR over rows of
 * h(f) = mix(sum_j mix((j << 32) | f(j))), mix = SplitMix64's output step. */
dm_status dm_result_hash(const dm_result* r, uint64_t* hash_sum, uint64_t* hash_xor);
/* Scored results: the cost of each held row (device pointer owned by the
 * result, NULL when the run was not scored), and a host copy of the first
 * max_rows costs (DM_ERR_INVALID_ARG when not scored). */
const uint64_t* dm_result_device_costs(const dm_result* r);
dm_status dm_result_copy_costs(const dm_result* r, uint64_t* dst, int64_t max_rows);
dm_status dm_result_copy_to_host(const dm_result* r, int32_t* dst, int64_t max_rows);
/* Device-to-device copy of up to max_rows rows into caller memory, ordered on
 * `hip_stream` (NULL = the context stream); synchronizes before returning. */
dm_status dm_result_copy_to_device(const dm_result* r, int32_t* dst, int64_t max_rows,
                                   void* hip_stream);

typedef struct {
    int32_t n_steps;          /* join-and-filter iterations (Fig. 3(c)(f)) */
    int32_t retries;          /* re-runs after a capacity overflow */
    int32_t chunks;           /* root-range partitions used */
    int32_t reserved;
    int64_t step_rows[DM_MAX_PATTERN_VERTICES]; /* rows after each step */
    double plan_ms;           /* host decomposition time */
    double device_ms;         /* device time of joins + sort */
    int64_t bytes_moved;      /* algorithmic bytes: every table read once + written once */
    /* filled when dm_plan_opts.profile = 1 (HIP events around each launch): */
    int32_t join_launches;    /* expand-join-filter kernel launches */
    int32_t sort_launches;
    double join_ms;           /* device time from the first join launch's start to the last one's end
                                 (one event pair: the kernel boundaries between them are included) */
    double sort_ms;           /* summed device time of the canonicalization launches */
    int64_t join_bytes;       /* algorithmic bytes of the join launches (4 * (c_in*n_in + c_out*n_out)) */
    int64_t sort_bytes;       /* algorithmic bytes of the sort (8 * width * rows) */
} dm_run_stats;

dm_status dm_result_stats(const dm_result* r, dm_run_stats* out);
void dm_result_free(dm_result* r);

/* The counts and launch accounting of n results at once (a batch's results,
 * a server's completions), one call instead of several per result. */
typedef struct {
    int64_t total;            /* dm_result_total */
    int64_t rows;             /* dm_result_rows */
    double join_ms;           /* the dm_run_stats fields of the same names */
    double sort_ms;
    int64_t join_bytes;
    int64_t sort_bytes;
    int32_t join_launches;
    int32_t sort_launches;
} dm_result_summary;

/* rs: host array of n result handles (none NULL), out: host array of n
 * summaries, both owned by the caller.  Errors: DM_ERR_INVALID_ARG (NULL
 * array, n < 0 or a NULL handle; out is then unspecified). */
dm_status dm_result_summaries(dm_result* const* rs, int32_t n, dm_result_summary* out);
/* dm_result_free on each of the n handles of the host array rs (NULL
 * entries are skipped); the array itself stays the caller's. */
void dm_result_free_many(dm_result* const* rs, int32_t n);

/* Served form: a request loop that keeps the data graph resident and runs
 * queries continuously on several streams (one worker each), in arrival
 * order, so that up to n_streams of them overlap on the device.  A query
 * predicted to build at most 4 MiB of intermediate tables is tiny: it takes
 * the tiny queries queued right behind it into one batch (one persistent
 * launch, at most max_batch queries and 32 MiB of predicted tables); every
 * other query runs alone through the per-step launches.  A query whose
 * predicted kept rows exceed 8 x mem_budget is refused at admission
 * (DM_ERR_BUDGET_EXCEEDED from dm_server_wait); one that passes the budget
 * while it runs fails the same way. */
typedef struct {
    int32_t n_streams;       /* concurrent batches in flight (default 2) */
    int32_t max_batch;       /* patterns per batch launch (default 64) */
    int64_t mem_budget;      /* bytes of predicted tables per batch, and each query's own
                                mem_budget and result_mb (default 8 GiB): a query whose result
                                exceeds it fails with DM_ERR_BUDGET_EXCEEDED.  The server holds
                                at most n_streams x mem_budget of tables. */
    int32_t max_queue;       /* pending requests before submit returns DM_ERR_BUSY (default 65536) */
} dm_server_opts;

dm_status dm_server_start(dm_datagraph* dg, const dm_server_opts* opts, dm_server** out);
/* Queue a pattern query (copied).  *ticket identifies it for dm_server_wait. */
dm_status dm_server_submit(dm_server* s, const dm_graph_desc* gp, int64_t max_embeddings,
                           uint64_t* ticket);
/* Wait up to timeout_ms (<0 = forever) for a ticket; DM_ERR_TIMEOUT if not done.
 * On DM_OK the caller owns *out.  A query's own failure is returned here. */
dm_status dm_server_wait(dm_server* s, uint64_t ticket, int32_t timeout_ms, dm_result** out);
/* Wait up to timeout_ms (<0 = forever) for any submitted query to finish
 * (in completion order; tickets already taken by dm_server_wait are passed
 * over); DM_ERR_TIMEOUT if none does.  On DM_OK, *ticket names the query and
 * *status is its own outcome: DM_OK with *out owned by the caller, or the
 * query's failure (e.g. DM_ERR_BUDGET_EXCEEDED) with *out NULL and the message
 * in dm_last_error().  One blocking call per completion: a caller collecting
 * results needs no polling. */
dm_status dm_server_wait_any(dm_server* s, int32_t timeout_ms, uint64_t* ticket, dm_result** out,
                             dm_status* status);
/* Stop accepting, finish in-flight work, free the server. */
dm_status dm_server_stop(dm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* DMOTIF_H */
