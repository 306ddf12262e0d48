// HIP kernels for gfx950 (wave64).  Everything here is integer table work:
// joins, filters, compaction, sorting and graph ingest.  None of it is a dense
// contraction, so nothing uses MFMA; the kernels are bound by HBM bandwidth
// (large tables) or by launch latency (small ones).
#include <algorithm>
#include <climits>
#include <type_traits>

#include "dm_device.hpp"

namespace dm {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Output-table store, coherent at agent scope: the value goes through to the
// point every XCD reads from instead of sitting dirty in this XCD's L2, so the
// tile's release fence has no table lines left to write back.
__device__ __forceinline__ void st_out(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back word: [epoch:14 | flag:2 | value:48]; flag 1 = tile aggregate,
// 2 = inclusive prefix.  A word from another epoch reads as "not ready".
constexpr uint64_t kValMask = (1ull << 48) - 1;
__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint32_t flag, uint64_t v) {
    return ((uint64_t)epoch << 50) | ((uint64_t)flag << 48) | (v & kValMask);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t ld_rlx_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The context's cancel word lives in host memory written by the host.
__device__ __forceinline__ uint32_t ld_sys_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Give up a wait (one lane calls this): the first wait of the run to give up
// sets the abort word and writes the record; later ones only leave.
__device__ void wait_give_up(const WaitCtl& w, int32_t reason, int32_t pattern, int32_t step, int32_t ntiles,
                             int64_t tile, int64_t spins, uint64_t ticks, int32_t claimed, int32_t finished) {
    if (atomicCAS(w.abort, 0u, (uint32_t)reason) != 0u) return;
    WaitDiag* d = w.diag;
    d->reason = reason;
    d->pattern = pattern;
    d->step = step;
    d->ntiles = ntiles;
    d->tile = tile;
    d->spins = spins;
    d->ticks = (int64_t)ticks;
    d->claimed = claimed;
    d->finished = finished;
    __threadfence();
}

// Decoupled look-back (single-pass chained scan) executed by one full wave.
// Tiles are claimed in ticket order by running workgroups, so every
// predecessor of `tile` is owned by a workgroup that is already running and
// publishes its aggregate before it waits itself: the wait ends.  It is
// bounded all the same (see WaitCtl): after `w.limit` wall-clock ticks, or
// once the run's abort word or the context's cancel word is set, it gives up
// and returns -1 (the caller then writes nothing).  Else returns the
// exclusive prefix.
__device__ int64_t lookback_wave(uint64_t* status, uint32_t epoch, int64_t tile, uint64_t agg, int lane,
                                 const WaitCtl& w, int32_t pattern, int32_t step) {
    if (tile == 0) {
        if (lane == 0) st_relaxed(&status[0], lb_pack(epoch, 2, agg));
        return 0;
    }
    if (lane == 0) st_relaxed(&status[tile], lb_pack(epoch, 1, agg));
    uint64_t excl = 0;
    int64_t j = tile - 1;
    int64_t spins = 0;
    uint64_t t0 = 0;
    for (;;) {
        const int64_t idx = j - lane;
        uint32_t flag = 2;
        uint64_t val = 0;
        if (idx >= 0) {
            const uint64_t s = ld_relaxed(&status[idx]);
            flag = ((uint32_t)(s >> 50) == epoch) ? (uint32_t)((s >> 48) & 3u) : 0u;
            val = s & kValMask;
        }
        const uint64_t pm = __ballot(flag == 2);
        const uint64_t zm = __ballot(flag == 0);
        const int p = pm ? (__ffsll((long long)pm) - 1) : 63;
        const uint64_t range = (p == 63) ? ~0ull : ((2ull << p) - 1ull);
        if (zm & range) {
            // a predecessor is not ready: bounded wait
            spins++;
            int stop = ld_rlx_u32(w.abort) != 0u ? WAIT_LOOKBACK : 0;
            if (!stop && (spins & 63) == 0) {
                const uint64_t now = wall_clock64();
                if (t0 == 0) {
                    t0 = now;
                } else if (now - t0 > w.limit) {
                    if (lane == 0) wait_give_up(w, WAIT_LOOKBACK, pattern, step, 0, tile, spins, now - t0, 0, 0);
                    stop = WAIT_LOOKBACK;
                }
                if (!stop && (spins & 255) == 0 && w.cancel && ld_sys_u32(w.cancel) != 0u) {
                    if (lane == 0) wait_give_up(w, WAIT_CANCEL, pattern, step, 0, tile, spins, now - t0, 0, 0);
                    stop = WAIT_CANCEL;
                }
            }
            if (__shfl(stop, 0, 64)) return -1;
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum_u64(lane <= p ? val : 0ull);
        if (pm) break;
        j -= 64;
    }
    if (lane == 0) st_relaxed(&status[tile], lb_pack(epoch, 2, excl + agg));
    return (int64_t)excl;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ bool adjacent(const GraphDev& g, int32_t u, int32_t v) {
    if (g.bitmap) {
        const uint32_t w = g.bitmap[(size_t)u * (size_t)g.words_per_row + (size_t)(v >> 5)];
        return (w >> (v & 31)) & 1u;
    }
    int32_t lo = g.row_ptr[u], hi = g.row_ptr[u + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t c = g.col[mid];
        if (c == v) return true;
        if (c < v) lo = mid + 1; else hi = mid;
    }
    return false;
}

// Cost of data edge {x, y} (an edge of the graph): ecost at y's CSR position in x's list.
__device__ __forceinline__ uint32_t edge_cost(const GraphDev& g, const uint32_t* ecost, int32_t x, int32_t y) {
    int32_t lo = g.row_ptr[x], hi = g.row_ptr[x + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t c = g.col[mid];
        if (c == y) return ecost[mid];
        if (c < y) lo = mid + 1; else hi = mid;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// expand-join-filter (one iteration of the join-and-filter loop)
// ---------------------------------------------------------------------------
//
// One tile = BLOCK consecutive input rows, one row per thread.  The row's
// values are staged in LDS (odd row stride, so lanes reading different rows
// hit different banks); a 128- or 256-bit summary of the row's values in
// registers settles most injectivity tests without the row scan.  On graphs
// with no more vertices than the summary has bits it is the exact vertex set
// (bit = vertex id), so a hit means a repeat and no test scans the row.  Candidates come from the motif
// table's direct-address index; survivors are counted, the tile's output
// offset comes from the look-back chain, and rows are written in input order
// with coalesced column stores.

// NW (2 or 4) 64-bit words, kept as named members so they stay in
// registers; bit of x = the top log2(64 NW) bits of x * mul.  EXACT: on
// graphs of at most 64 NW vertices mul = 2^(32 - log2(64 NW)), so bit = x.
template <int NW, bool EXACT>
struct Bloom {
    static constexpr int kLogBits = NW == 4 ? 8 : 7;
    static constexpr uint32_t kHashMul = 0x9E3779B1u;
    uint64_t w0, w1, w2, w3;
    uint32_t mul;
    bool exact;
    __device__ __forceinline__ void init(int32_t n_vertices) {
        w0 = w1 = w2 = w3 = 0;
        exact = EXACT && n_vertices <= 64 * NW;
        mul = exact ? (1u << (32 - kLogBits)) : kHashMul;
    }
    __device__ __forceinline__ uint32_t bit(int32_t x) const {
        return ((uint32_t)x * (EXACT ? mul : kHashMul)) >> (32 - kLogBits);
    }
    __device__ __forceinline__ void add(int32_t x) {
        const uint32_t b = bit(x), q = b >> 6;
        const uint64_t m = 1ull << (b & 63);
        w0 |= q == 0 ? m : 0ull;
        w1 |= q == 1 ? m : 0ull;
        if (NW == 4) {
            w2 |= q == 2 ? m : 0ull;
            w3 |= q == 3 ? m : 0ull;
        }
    }
    __device__ __forceinline__ bool maybe(int32_t x) const {
        const uint32_t b = bit(x), q = b >> 6;
        uint64_t v = q == 0 ? w0 : w1;
        if (NW == 4) v = q == 2 ? w2 : (q == 3 ? w3 : v);
        return (v >> (b & 63)) & 1ull;
    }
    __device__ __forceinline__ bool is_exact() const { return EXACT && exact; }
};

template <int NV>
__device__ __forceinline__ int32_t pick_new(const int32_t (&nv)[NV], int t) {
    int32_t r = -1;
#pragma unroll
    for (int i = 0; i < NV; i++) r = (i == t) ? nv[i] : r;
    return r;
}

// Does motif row m extend this thread's input row (in LDS at `my`) into a
// valid partial embedding?  Further join keys, injectivity of the new values
// against the row, and the step's explicit edge checks.
// NV: the most new values a step of this instantiation adds (registers per
// candidate); steps adding more than kNarrowNew values use the wide one.
// NEQ: further join keys loaded together with the new values (the rest are
// loaded and tested one at a time).
template <int NV, int NEQ, class BL>
__device__ __forceinline__ bool ejf_accept(const EjfArgs& a, const int32_t* my, const BL& bl, int32_t m,
                                           int32_t (&nv)[NV]) {
    const StepDesc& st = a.st;
    const int c_in = st.c_in;
    if (st.motif >= 0) {
        // issue every load of this candidate before the first compare
        const int32_t* tb = a.tbl.base + (int64_t)m * a.tbl.rstride;
        const int64_t ts = a.tbl.stride;
        const int n_new = st.n_new, n_eq = st.n_eq;
        int32_t ev[NEQ > 0 ? NEQ : 1];
#pragma unroll
        for (int e = 0; e < NEQ; e++)
            if (e < n_eq) ev[e] = tb[(int64_t)st.eq_pos[e] * ts];
#pragma unroll
        for (int t = 0; t < NV; t++)
            if (t < n_new) nv[t] = tb[(int64_t)st.new_pos[t] * ts];
#pragma unroll
        for (int e = 0; e < NEQ; e++)
            if (e < n_eq && ev[e] != my[st.eq_col[e]]) return false;
        for (int e = NEQ; e < n_eq; e++)
            if (tb[(int64_t)st.eq_pos[e] * ts] != my[st.eq_col[e]]) return false;
#pragma unroll
        for (int t = 0; t < NV; t++) {
            if (t < n_new) {
                const int32_t x = nv[t];
                if (bl.maybe(x)) {
                    if (bl.is_exact()) return false;
                    for (int c = 0; c < c_in; c++)
                        if (my[c] == x) return false;
                }
            }
        }
    }
    for (int e = 0; e < st.n_edge; e++) {
        const int ca = st.edge_a[e], cb = st.edge_b[e];
        const int32_t va = ca < c_in ? my[ca] : pick_new(nv, ca - c_in);
        const int32_t vb = cb < c_in ? my[cb] : pick_new(nv, cb - c_in);
        if (!adjacent(a.g, va, vb)) return false;
    }
    if (a.induced && st.motif >= 0) {
        // induced variant: every data neighbour of a new vertex that the row
        // already holds must sit in a column whose pattern vertex is adjacent
        for (int t = 0; t < st.n_new; t++) {
            const int32_t x = pick_new(nv, t);
            const uint64_t m0 = st.padj[t][0], m1 = st.padj[t][1];
            for (int32_t i = a.g.row_ptr[x], e = a.g.row_ptr[x + 1]; i < e; i++) {
                const int32_t w = a.g.col[i];
                int c = -1;
                if (bl.maybe(w))
                    for (int q = 0; q < c_in; q++)
                        if (my[q] == w) c = q;
                for (int q = 0; q < t; q++)
                    if (pick_new(nv, q) == w) c = c_in + q;
                if (c >= 0 && !(((c < 64 ? m0 : m1) >> (c & 63)) & 1ull)) return false;
            }
        }
    }
    return true;
}

// Per-step constants of the per-launch candidate test, staged in LDS once
// per workgroup: each candidate then reads them with a few broadcast loads
// instead of holding them in scalar registers across the whole kernel.
struct AcceptLds {
    int64_t noff[kMaxMotif];  // element offset of new value t in a motif row; past the
                              // step's last new value, that value's again
    int64_t eoff[kMaxMotif];  // element offset of further join key e
    int32_t eqcol[kMaxMotif]; // the input column it must equal
    int32_t e0;               // first further key to test (1: the first one holds by
                              // construction, the candidates being its run)
};

// Stage the step's constants (threads 0..kMaxMotif-1; a barrier follows before use).
__device__ __forceinline__ void accept_lds_fill(const EjfArgs& a, AcceptLds& k) {
    const int t = threadIdx.x;
    if (t < kMaxMotif) {
        const StepDesc& st = a.st;
        const int nn = st.motif >= 0 ? st.n_new : 0;
        const int64_t ts = a.tbl.stride;
        k.noff[t] = nn > 0 ? (int64_t)st.new_pos[t < nn ? t : nn - 1] * ts : 0;
        k.eoff[t] = t < st.n_eq ? (int64_t)st.eq_pos[t] * ts : 0;
        k.eqcol[t] = t < st.n_eq ? st.eq_col[t] : 0;
        if (t == 0)
            k.e0 = (st.motif >= 0 && st.n_eq > 0 && a.tbl.pair_offs && a.tbl.sorted_by == st.eq_pos[0] + 1) ? 1 : 0;
    }
}

// The test of ejf_accept for the per-launch form, written so that every
// candidate runs the same instructions: all NV value loads unconditionally
// (an instantiation's NV is the step's new-value count rounded up to the
// next instantiated size; the extra slots repeat the last new value, which
// changes no test), outcomes as predicates rather than early exits, and the
// row scan that settles the summary's maybe-hits run once for the wave when
// any lane needs it, as one compare per (row value, new value) pair.  Only
// the edge and induced checks, after that, still leave early.
template <int NV, class BL>
__device__ __forceinline__ bool ejf_accept_flat(const EjfArgs& a, const AcceptLds& k, const int32_t* my,
                                                const BL& bl, int32_t m, int32_t (&nv)[NV]) {
    const StepDesc& st = a.st;
    const int c_in = st.c_in;
    bool ok = true;
    if (st.motif >= 0) {
        const int32_t* tb = a.tbl.base + (int64_t)m * a.tbl.rstride;
#pragma unroll
        for (int t = 0; t < NV; t++) nv[t] = tb[k.noff[t]];
        for (int e = k.e0; e < st.n_eq; e++) ok &= tb[k.eoff[e]] == my[k.eqcol[e]];
        bool hit = false;
#pragma unroll
        for (int t = 0; t < NV; t++) hit |= bl.maybe(nv[t]);
        if (bl.is_exact()) {
            ok &= !hit;
        } else if (__any(ok && hit)) {
            // zero iff some row value equals some new value (vector ALU only:
            // a minimum of differences, no per-compare lane masks)
            uint32_t d = ~0u;
            for (int c = 0; c < c_in; c++) {
                const uint32_t v = (uint32_t)my[c];
#pragma unroll
                for (int t = 0; t < NV; t++) d = min(d, v ^ (uint32_t)nv[t]);
            }
            ok &= d != 0u;
        }
    }
    if (st.n_edge > 0 || (a.induced && st.motif >= 0)) {
        if (!ok) return false;
        for (int e = 0; e < st.n_edge; e++) {
            const int ca = st.edge_a[e], cb = st.edge_b[e];
            const int32_t va = ca < c_in ? my[ca] : pick_new(nv, ca - c_in);
            const int32_t vb = cb < c_in ? my[cb] : pick_new(nv, cb - c_in);
            if (!adjacent(a.g, va, vb)) return false;
        }
        if (a.induced && st.motif >= 0) {
            for (int t = 0; t < st.n_new; t++) {
                const int32_t x = pick_new(nv, t);
                const uint64_t m0 = st.padj[t][0], m1 = st.padj[t][1];
                for (int32_t i = a.g.row_ptr[x], e = a.g.row_ptr[x + 1]; i < e; i++) {
                    const int32_t w = a.g.col[i];
                    int c = -1;
                    if (bl.maybe(w))
                        for (int q = 0; q < c_in; q++)
                            if (my[q] == w) c = q;
                    for (int q = 0; q < t; q++)
                        if (pick_new(nv, q) == w) c = c_in + q;
                    if (c >= 0 && !(((c < 64 ? m0 : m1) >> (c & 63)) & 1ull)) return false;
                }
            }
        }
    }
    return ok;
}

// Candidate-parallel tiles hold at most this many 64-candidate chunks per
// wave, and test rows of at most kCpScanCols values by the row scan alone.
constexpr int kCpChunks = 32;
constexpr int kCpScanCols = 16;

template <int BLOCK>
struct CpShared {
    int32_t mdelta[BLOCK];  // each row's first motif row minus its first candidate number
    uint64_t bl[BLOCK][2];  // each row's summary words (rows wider than kCpScanCols)
    uint64_t inner[BLOCK];  // count+hash mode: each row's inner hash
    uint64_t mask[BLOCK / 64][kCpChunks];       // survivors of each 64-candidate chunk
    uint8_t owner[BLOCK / 64][64 * kCpChunks];  // the row (lane) of each candidate of the wave
};
struct NoCpShared {};

// CP: with the candidate-parallel part (kernels that have that form only,
// so the others keep their smaller LDS footprint).
template <int BLOCK, bool CP = false>
struct TileShared {
    static constexpr int CH = 8 * BLOCK;  // output rows staged per write pass
    int64_t base;
    int32_t total;
    int32_t wsum[BLOCK / 64];
    int32_t wexcl[BLOCK / 64];
    union {
        struct {
            int32_t mrow[CH];   // motif row of each staged output row
            uint8_t src[CH];    // input row (lane of the tile) of each staged output row
        } st;
        std::conditional_t<CP, CpShared<BLOCK>, NoCpShared> cp;
    };
};

// Stands in for the row summary where the row scan alone decides: every
// value may be in the row.
struct NoSummary {
    __device__ __forceinline__ bool maybe(int32_t) const { return true; }
    __device__ __forceinline__ bool is_exact() const { return false; }
};

// Row stride (in int32) of the LDS row tile for c columns: odd, >= c.
__host__ __device__ __forceinline__ int row_stride(int c) { return c | 1; }

// Output offset of each wave's first row in this tile: wave totals scanned
// across the workgroup, the tile's offset from the look-back chain.  Leaves
// sh.base / sh.total (both 0 when the look-back gave up) and sh.wexcl.
template <int BLOCK, class SH>
__device__ __forceinline__ void tile_offsets(const EjfArgs& a, int64_t tile, int64_t n_tiles, SH& sh,
                                             int32_t wave_total) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (lane == 0) sh.wsum[wid] = wave_total;
    __syncthreads();
    if (wid == 0) {
        int32_t w = lane < NW ? sh.wsum[lane] : 0;
        int32_t wi = w;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            const int32_t y = __shfl_up(wi, o, 64);
            if (lane >= o) wi += y;
        }
        if (lane < NW) sh.wexcl[lane] = wi - w;
        const int32_t total = __shfl(wi, NW - 1, 64);
        const int64_t excl = lookback_wave(a.status, a.epoch, tile, (uint64_t)total, lane, a.w, a.diag_pattern,
                                           a.diag_step);
        if (lane == 0) {
            if (excl < 0) {
                // the look-back gave up (the run is being aborted): write nothing
                sh.base = 0;
                sh.total = 0;
            } else {
                sh.base = excl;
                sh.total = total;
                if (tile == n_tiles - 1) *a.n_out = excl + total;
                if (excl + total > a.out_cap) *a.overflow = 1;
            }
        }
    }
    __syncthreads();
}

// Candidate-parallel form of a tile, for steps whose rows have many
// candidates of uneven number (a key group of a large motif table, the run of
// a two-key join).  Looping over its own candidates, a lane would keep its
// wave as long as the row with the most; here the candidates of a wave's 64
// rows are numbered consecutively (a scan of their counts; each row writes
// its lane into the owner byte of its candidates) and the wave tests them 64
// at a time, lane i taking candidate 64 j + i.  Consecutive lanes read
// consecutive motif rows.  Survivors of each group of 64 are kept as one
// ballot word in LDS; after the tile's offset is known, each lane writes its
// survivor's whole row, at the survivor's rank among the tile's, so the output
// is the row-by-row one.  Returns false (the whole workgroup alike, before any
// output) when some wave has more candidates than its owner bytes hold; the
// caller then runs the row-per-lane form.
template <int BLOCK, int NV>
__device__ __forceinline__ bool ejf_tile_cp(const EjfArgs& a, const AcceptLds& ka, int64_t tile, int64_t n_tiles,
                                            TileShared<BLOCK, true>& sh, const int32_t* rows,
                                            const Bloom<2, false>& bl, int32_t lo, int32_t cnt, uint64_t inner_old,
                                            uint64_t& h_cnt, uint64_t& h_sum, uint64_t& h_xor) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const StepDesc& st = a.st;
    const int c_in = st.c_in;
    const int RS = row_stride(c_in);
    const bool hash = a.mode == EJF_HASH;
    int32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    const int32_t wtot = __builtin_amdgcn_readfirstlane(__shfl(x, 63, 64));  // wave-uniform
    const bool fits = wtot <= 64 * kCpChunks;
    const int32_t c0 = x - cnt;
    uint8_t* own = sh.cp.owner[wid];
    if (fits)
        for (int32_t q = 0; q < cnt; q++) own[c0 + q] = (uint8_t)lane;
    sh.cp.mdelta[tid] = lo - c0;
    sh.cp.bl[tid][0] = bl.w0;
    sh.cp.bl[tid][1] = bl.w1;
    sh.cp.inner[tid] = inner_old;
    if (__syncthreads_or(!fits)) return false;

    const int w0 = wid * 64;
    const int nch = (wtot + 63) >> 6;
    const int n_new = st.n_new;
    const bool scan_only = c_in <= kCpScanCols;
    auto accept = [&](int r, int32_t m, int32_t (&nv)[NV]) -> bool {
        const int32_t* orow = rows + (w0 + r) * RS;
        bool ok;
        if (scan_only) {
            ok = ejf_accept_flat<NV>(a, ka, orow, NoSummary{}, m, nv);
        } else {
            Bloom<2, false> ob;
            ob.init(a.g.n);
            ob.w0 = sh.cp.bl[w0 + r][0];
            ob.w1 = sh.cp.bl[w0 + r][1];
            ok = ejf_accept_flat<NV>(a, ka, orow, ob, m, nv);
        }
        if (ok && hash) {
            uint64_t inner = sh.cp.inner[w0 + r];
#pragma unroll
            for (int t = 0; t < NV; t++)
                if (t < n_new) inner += mix64(((uint64_t)a.pv[c_in + t] << 32) | (uint32_t)nv[t]);
            const uint64_t h = mix64(inner);
            h_cnt++;
            h_sum += h;
            h_xor ^= h;
        }
        return ok;
    };
    int32_t surv = 0;
    for (int j = 0; j < nch; j++) {
        const int32_t c = j * 64 + lane;
        bool ok = false;
        if (c < wtot) {
            int32_t nv[NV];
            const int r = own[c];
            ok = accept(r, c + sh.cp.mdelta[w0 + r], nv);
        }
        if (!hash) {
            const uint64_t mk = __ballot(ok);
            if (lane == 0) sh.cp.mask[wid][j] = mk;
            surv += __popcll(mk);
        }
    }
    if (hash) return true;  // nothing written: the tile's LDS may be reused at once

    tile_offsets<BLOCK>(a, tile, n_tiles, sh, surv);
    if (sh.total == 0) return true;
    const int64_t base = sh.base + sh.wexcl[wid];
    const int64_t os = a.out_stride;
    int64_t cand_acc = 0;
    int32_t pre = 0;
    for (int j = 0; j < nch; j++) {
        const uint64_t mk = sh.cp.mask[wid][j];
        if ((mk >> lane) & 1ull) {
            const int64_t orow = base + pre + __popcll(mk & ((1ull << lane) - 1ull));
            if (orow < a.out_cap) {
                const int32_t c = j * 64 + lane;
                const int r = own[c];
                const int32_t m = c + sh.cp.mdelta[w0 + r];
                const int32_t* prow = rows + (w0 + r) * RS;
                const int32_t* tb = a.tbl.base + (int64_t)m * a.tbl.rstride;
                int32_t nv[NV];
#pragma unroll
                for (int t = 0; t < NV; t++) nv[t] = tb[ka.noff[t]];
                int32_t* dst = a.out + orow;
                for (int cc = 0; cc < c_in; cc++, dst += os) *dst = prow[cc];
#pragma unroll
                for (int t = 0; t < NV; t++)
                    if (t < n_new) dst[t * os] = nv[t];
                if (a.next_cand) {
                    const int nk = a.next_key_col;
                    if (nk < 0) {
                        cand_acc += 1;
                    } else {
                        const int32_t kv = nk < c_in ? prow[nk] : pick_new(nv, nk - c_in);
                        cand_acc += a.next_offs[kv + 1] - a.next_offs[kv];
                    }
                }
            }
        }
        pre += __popcll(mk);
    }
    if (a.next_cand) {
        const uint64_t w = wave_sum_u64((uint64_t)cand_acc);
        if (lane == 0 && w) atomicAdd((unsigned long long*)a.next_cand, (unsigned long long)w);
    }
    return true;
}

// SCORE: the layout-cost column is carried (scored runs only; the batched
// form never scores, so its instantiation carries no cost code).
// LAT: the latency-bound persistent form.  Its tiles hand tables to other
// XCDs through a release per tile, so outputs are stored coherently at agent
// scope (nothing dirty left in L2 for the release to write back), and its
// summary is 256 bits wide (exact up to 256 vertices).  The per-launch form
// is throughput-bound on large tables: plain stores, 128 bits.
// CP: steps marked for the candidate-parallel form try it first (ejf_tile_cp).
template <int BLOCK, int NV, bool SCORE, bool LAT, bool CP = false>
__device__ __forceinline__ void ejf_tile(const EjfArgs& a, const AcceptLds* ka, int64_t tile, int64_t n_in,
                                         int64_t n_tiles, TileShared<BLOCK, CP>& sh, int32_t* rows, uint64_t& h_cnt,
                                         uint64_t& h_sum, uint64_t& h_xor) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const StepDesc& st = a.st;
    const int c_in = st.c_in;
    const int RS = row_stride(c_in);
    const int64_t row = tile * BLOCK + tid;
    const bool valid = row < n_in;
    int32_t* my = rows + tid * RS;
    Bloom<LAT ? 4 : 2, LAT> bl;
    bl.init(a.g.n);
    constexpr int NEQ = LAT ? 4 : 0;
    constexpr int RCH = LAT ? 16 : 8;  // input columns loaded per round
    uint64_t inner_old = 0;
    const bool hash = a.mode == EJF_HASH;
    // the latency-bound form keeps its early-exit test with further keys
    // loaded up front; the per-launch form the flat one (per-step constants
    // in LDS at ka)
    auto accept = [&](int32_t m, int32_t (&v)[NV]) -> bool {
        if constexpr (LAT) return ejf_accept<NV, NEQ>(a, my, bl, m, v);
        else return ejf_accept_flat<NV>(a, *ka, my, bl, m, v);
    };
    if (valid) {
        if (a.in) {
            const int32_t* src = a.in + (a.in_row0 ? *a.in_row0 : 0) + row;
            const int64_t is = a.in_stride;
            for (int c0 = 0; c0 < c_in; c0 += RCH) {
                int32_t tv[RCH];
#pragma unroll
                for (int j = 0; j < RCH; j++)
                    if (c0 + j < c_in) tv[j] = src[(int64_t)(c0 + j) * is];
#pragma unroll
                for (int j = 0; j < RCH; j++) {
                    if (c0 + j < c_in) {
                        my[c0 + j] = tv[j];
                        bl.add(tv[j]);
                        if (hash) inner_old += mix64(((uint64_t)a.pv[c0 + j] << 32) | (uint32_t)tv[j]);
                    }
                }
            }
        } else {
            const int32_t x = a.id_begin + (int32_t)row;
            my[0] = x;
            bl.add(x);
            if (hash) inner_old += mix64(((uint64_t)a.pv[0] << 32) | (uint32_t)x);
        }
    }
    int32_t lo = 0, hi = 0;
    if (valid) {
        if (st.motif >= 0) {
            const int32_t key = my[st.key_col];
            lo = a.tbl.offs[key];
            hi = a.tbl.offs[key + 1];
            if (!LAT && st.n_eq > 0 && a.tbl.sorted_by == st.eq_pos[0] + 1) {
                // the key group is ordered by the first further key's position:
                // keep only its run equal to this row's value (the rest fail that
                // key anyway, and the test below still checks every candidate)
                const int32_t want = my[st.eq_col[0]];
                if (a.tbl.pair_offs) {
                    // the group's distinct values of that position, with the
                    // row each run starts at: one short search, few lines
                    const int32_t pl = a.tbl.pair_offs[key], ph = a.tbl.pair_offs[key + 1];
                    int32_t l = pl, h = ph;
                    while (l < h) {
                        const int32_t mid = (l + h) >> 1;
                        if (a.tbl.pair_far[mid] < want) l = mid + 1; else h = mid;
                    }
                    if (l < ph && a.tbl.pair_far[l] == want) {
                        lo = a.tbl.pair_start[l];
                        hi = l + 1 < ph ? a.tbl.pair_start[l + 1] : hi;
                    } else {
                        lo = hi;
                    }
                } else if (hi - lo > 16 && hi - lo <= a.tbl.sorted_max) {
                    const int32_t* sc = a.tbl.base + (int64_t)st.eq_pos[0] * a.tbl.stride;
                    const int64_t rs = a.tbl.rstride;
                    int32_t l = lo, h = hi;
                    while (l < h) {
                        const int32_t mid = (l + h) >> 1;
                        if (sc[mid * rs] < want) l = mid + 1; else h = mid;
                    }
                    int32_t e = l;
                    h = hi;
                    while (e < h) {
                        const int32_t mid = (e + h) >> 1;
                        if (sc[mid * rs] <= want) e = mid + 1; else h = mid;
                    }
                    lo = l;
                    hi = e;
                }
            }
        } else {
            hi = 1;  // filter-only step: the row itself is the one candidate
        }
    }
    if constexpr (CP && !LAT && !SCORE) {
        if (ejf_tile_cp<BLOCK, NV>(a, *ka, tile, n_tiles, sh, rows, bl, lo, valid ? hi - lo : 0, inner_old,
                                                 h_cnt, h_sum, h_xor))
            return;
    }
    int32_t nv[NV];
#pragma unroll
    for (int t = 0; t < NV; t++) nv[t] = -1;

    if (hash) {
        for (int32_t m = lo; m < hi; m++) {
            if (!accept(m, nv)) continue;
            uint64_t inner = inner_old;
#pragma unroll
            for (int t = 0; t < NV; t++)
                if (t < st.n_new) inner += mix64(((uint64_t)a.pv[c_in + t] << 32) | (uint32_t)nv[t]);
            const uint64_t h = mix64(inner);
            h_cnt++;
            h_sum += h;
            h_xor ^= h;
        }
        return;  // no lane read another lane's row: the tile can be reused at once
    }

    uint64_t mask = 0;
    int32_t cnt = 0;
    if (LAT && st.motif >= 0 && st.n_eq > 0) {
        // Most candidates fail the first further join key: test it for eight
        // candidates per round of loads, then run the full test on the rest.
        const int32_t* kcol = a.tbl.base + (int64_t)st.eq_pos[0] * a.tbl.stride;
        const int64_t krs = a.tbl.rstride;
        const int32_t want = my[st.eq_col[0]];
        for (int32_t m0 = lo; m0 < hi; m0 += 8) {
            int32_t k8[8];
#pragma unroll
            for (int j = 0; j < 8; j++) k8[j] = (m0 + j < hi) ? kcol[(int64_t)(m0 + j) * krs] : ~want;
            uint32_t pm = 0;
#pragma unroll
            for (int j = 0; j < 8; j++) pm |= (uint32_t)(k8[j] == want) << j;
            while (pm) {
                const int j = __ffs((int)pm) - 1;
                pm &= pm - 1;
                const int32_t m = m0 + j;
                if (accept(m, nv)) {
                    if (m - lo < 64) mask |= 1ull << (m - lo);
                    cnt++;
                }
            }
        }
    } else {
        for (int32_t m = lo; m < hi; m++) {
            if (accept(m, nv)) {
                if (m - lo < 64) mask |= 1ull << (m - lo);
                cnt++;
            }
        }
    }
    // block-wide exclusive scan of per-row survivor counts
    int32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    tile_offsets<BLOCK>(a, tile, n_tiles, sh, __shfl(x, 63, 64));
    // Write phase: survivors are staged in LDS in output order as (input
    // lane, motif row); then each thread assembles whole output rows (parent
    // values from the LDS row tile, new values from the motif table) and
    // writes them column by column, so every store of a wave covers
    // consecutive elements of one column.
    constexpr int CH = TileShared<BLOCK>::CH;
    const int32_t local0 = sh.wexcl[wid] + (x - cnt);
    const int32_t total = sh.total;
    const int64_t base = sh.base;
    const int n_new = st.motif >= 0 ? st.n_new : 0;
    // each thread's candidate cursor survives across passes, so every
    // candidate is visited once however many passes the tile needs
    int32_t m_cur = lo, r_cur = 0;
    int64_t cand_acc = 0;  // next step's candidates of the rows this thread writes
    for (int32_t w0 = 0; w0 < total; w0 += CH) {
        while (r_cur < cnt && m_cur < hi) {
            const int32_t li = local0 + r_cur;
            if (li >= w0 + CH) break;  // belongs to a later pass
            const int32_t m = m_cur++;
            const bool ok = (m - lo < 64) ? (bool)((mask >> (m - lo)) & 1ull) : accept(m, nv);
            if (!ok) continue;
            sh.st.src[li - w0] = (uint8_t)tid;
            sh.st.mrow[li - w0] = m;
            r_cur++;
        }
        __syncthreads();
        const int32_t nrows = (total - w0 < CH) ? (total - w0) : CH;
        const int64_t obase = base + w0;
        for (int32_t o = tid; o < nrows; o += BLOCK) {
            const int64_t orow = obase + o;
            if (orow >= a.out_cap) break;
            const int32_t* prow = rows + sh.st.src[o] * RS;
            const int32_t m = sh.st.mrow[o];
            int32_t* dst = a.out + orow;
            const int64_t os = a.out_stride;
            {
                int32_t* d = dst;
                for (int c = 0; c < c_in; c++, d += os) {
                    if (LAT) st_out(d, prow[c]);
                    else *d = prow[c];
                }
            }
            const int32_t* tb = a.tbl.base + (int64_t)m * a.tbl.rstride;
            const int64_t ts = a.tbl.stride;
            if (n_new > 0) {
                for (int t0 = 0; t0 < n_new; t0 += 4) {
                    int32_t w4[4];
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        if (t0 + j < n_new) w4[j] = tb[(int64_t)st.new_pos[t0 + j] * ts];
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        if (t0 + j < n_new) {
                            if (LAT) st_out(dst + (int64_t)(c_in + t0 + j) * os, w4[j]);
                            else dst[(int64_t)(c_in + t0 + j) * os] = w4[j];
                        }
                }
            }
            if (SCORE && a.out_cost) {
                // layout cost: the parent's plus the new vertices' and the new edges'
                uint64_t cst = a.in ? a.in_cost[tile * BLOCK + sh.st.src[o]] : (uint64_t)a.vcost[prow[0]];
                for (int t = 0; t < n_new; t++) {
                    const int32_t x = tb[(int64_t)st.new_pos[t] * ts];
                    cst += a.vcost[x];
                    uint64_t m0 = st.padj[t][0], m1 = st.padj[t][1];
                    while (m0 | m1) {
                        int c;
                        if (m0) {
                            c = __ffsll((long long)m0) - 1;
                            m0 &= m0 - 1;
                        } else {
                            c = 64 + __ffsll((long long)m1) - 1;
                            m1 &= m1 - 1;
                        }
                        const int32_t y = c < c_in ? prow[c] : tb[(int64_t)st.new_pos[c - c_in] * ts];
                        cst += edge_cost(a.g, a.ecost, x, y);
                    }
                }
                a.out_cost[orow] = cst;
            }
            if (a.next_cand) {
                const int nk = a.next_key_col;
                if (nk < 0) {
                    cand_acc += 1;
                } else {
                    const int32_t kv = nk < c_in ? prow[nk] : tb[(int64_t)st.new_pos[nk - c_in] * ts];
                    cand_acc += a.next_offs[kv + 1] - a.next_offs[kv];
                }
            }
        }
        __syncthreads();  // other lanes' rows were read: the next tile may overwrite them only now
    }
    if (a.next_cand && total > 0) {
        const uint64_t w = wave_sum_u64((uint64_t)cand_acc);
        if (lane == 0 && w) atomicAdd((unsigned long long*)a.next_cand, (unsigned long long)w);
    }
}

template <int BLOCK>
__device__ void hash_flush(uint64_t* acc, uint64_t h_cnt, uint64_t h_sum, uint64_t h_xor, uint64_t (*red)[BLOCK / 64]) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        h_cnt += __shfl_xor(h_cnt, o, 64);
        h_sum += __shfl_xor(h_sum, o, 64);
        h_xor ^= __shfl_xor(h_xor, o, 64);
    }
    if (lane == 0) {
        red[0][wid] = h_cnt;
        red[1][wid] = h_sum;
        red[2][wid] = h_xor;
    }
    __syncthreads();
    if (tid == 0) {
        uint64_t c = 0, s = 0, xr = 0;
        for (int w = 0; w < NW; w++) {
            c += red[0][w];
            s += red[1][w];
            xr ^= red[2][w];
        }
        if (c) {
            atomicAdd((unsigned long long*)&acc[0], (unsigned long long)c);
            atomicAdd((unsigned long long*)&acc[1], (unsigned long long)s);
            atomicXor((unsigned long long*)&acc[2], (unsigned long long)xr);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int64_t clamp_rows(int64_t n, int64_t cap) { return n < 0 ? 0 : (n > cap ? cap : n); }

// One join-filter step over one table: workgroups claim tiles in ticket order
// until the input is exhausted.  Dynamic LDS: BLOCK * row_stride(c_in) int32.
template <int BLOCK, int NV, bool SCORE, bool CP>
__global__ __launch_bounds__(BLOCK, NV <= 6 ? 5 : 1) void ejf_kernel(const EjfArgs a) {
    extern __shared__ int32_t rows[];
    __shared__ TileShared<BLOCK, CP> sh;
    __shared__ AcceptLds ka;
    __shared__ int64_t s_tile;
    __shared__ uint64_t s_red[3][BLOCK / 64];
    const int tid = threadIdx.x;
    accept_lds_fill(a, ka);  // read after the barrier of the first claim
    const int64_t n_in = a.in ? clamp_rows(*a.n_in, a.in_cap) : (int64_t)a.id_count;
    const int64_t n_tiles = (n_in + BLOCK - 1) / BLOCK;
    uint64_t h_cnt = 0, h_sum = 0, h_xor = 0;
    // an earlier wait of the run gave up: its tables are incomplete, so this
    // step reads nothing (and claims nothing more)
    auto claim = [&]() -> int64_t {
        return ld_rlx_u32(a.w.abort) != 0u ? -1 : (int64_t)atomicAdd((unsigned long long*)a.ticket, 1ull);
    };
    for (;;) {
        if (tid == 0) s_tile = claim();
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile < 0) {
            if (a.mode == EJF_WRITE && blockIdx.x == 0 && tid == 0) *a.n_out = 0;
            break;
        }
        if (tile >= n_tiles) {
            if (a.mode == EJF_WRITE && tile == 0 && tid == 0) *a.n_out = 0;
            break;
        }
        ejf_tile<BLOCK, NV, SCORE, false, CP>(a, &ka, tile, n_in, n_tiles, sh, rows, h_cnt, h_sum, h_xor);
    }
    if (a.mode == EJF_HASH) hash_flush<BLOCK>(a.hash_acc, h_cnt, h_sum, h_xor, s_red);
}

int ejf_block_for(int c_in, int requested) {
    // the LDS row tile stays within ~34 KB: wide rows take smaller tiles
    const int cap = c_in <= 31 ? 256 : (c_in <= 63 ? 128 : 64);
    int b = requested > 0 ? requested : cap;
    return b > cap ? cap : b;
}

hipError_t launch_ejf(const EjfArgs& a, int block, int grid, hipStream_t s) {
    const int c = a.st.c_in;
    block = ejf_block_for(c, block);
    const size_t lds = sizeof(int32_t) * (size_t)block * row_stride(c);
#define DM_EJF_GO(B, NV, SC, CP) hipLaunchKernelGGL((ejf_kernel<B, NV, SC, CP>), dim3(grid), dim3(B), lds, s, a);
#define DM_EJF_LAUNCH(NV, SC, CP)                  \
    switch (block) {                               \
        case 64: DM_EJF_GO(64, NV, SC, CP) break;   \
        case 128: DM_EJF_GO(128, NV, SC, CP) break; \
        default: DM_EJF_GO(256, NV, SC, CP) break;  \
    }
#define DM_EJF_LAUNCH_CP(NV)      \
    if (cp) {                     \
        DM_EJF_LAUNCH(NV, false, true) \
    } else {                      \
        DM_EJF_LAUNCH(NV, false, false) \
    }
    // instantiations: the step's new values rounded up to 1, 2, 4, 6, 12 or
    // 18 (the test loads that many per candidate), each also in the
    // candidate-parallel form; scored runs (rare) take 12 or 18
    const int nn = a.st.motif >= 0 ? a.st.n_new : 0;
    const bool scored = a.out_cost != nullptr, cp = a.cand_par != 0;
    if (scored) {
        if (nn > kNarrowNew) {
            DM_EJF_LAUNCH(kMaxMotif, true, false)
        } else {
            DM_EJF_LAUNCH(kNarrowNew, true, false)
        }
    } else if (nn <= 1) {
        DM_EJF_LAUNCH_CP(1)
    } else if (nn <= 2) {
        DM_EJF_LAUNCH_CP(2)
    } else if (nn <= 4) {
        DM_EJF_LAUNCH_CP(4)
    } else if (nn <= 6) {
        DM_EJF_LAUNCH_CP(6)
    } else if (nn <= kNarrowNew) {
        DM_EJF_LAUNCH_CP(kNarrowNew)
    } else {
        DM_EJF_LAUNCH_CP(kMaxMotif)
    }
#undef DM_EJF_LAUNCH_CP
#undef DM_EJF_GO
#undef DM_EJF_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched form: one persistent launch runs every pattern's join steps
// ---------------------------------------------------------------------------
//
// Work unit = (pattern p, step s, tile t).  A pattern's step s becomes
// claimable once its step s-1 finished (ctl.stage == s); its tiles are
// claimed in ticket order from ctl.claim[s], so the order-preserving
// look-back of a tile only ever waits on tiles held by running workgroups.
// The workgroup that finishes the last tile of a step publishes the next
// step (or retires the pattern).  Every workgroup exits once all patterns
// are retired, so the grid always drains.

__device__ __forceinline__ int32_t ld_rlx_i32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel_i32(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// One tile = BLOCK rows; wave 0 finds and claims tiles for the workgroup.
// Dynamic LDS: BLOCK * row_stride(widest input) int32.
template <int BLOCK, int NV>
__global__ __launch_bounds__(BLOCK) void batch_kernel(const BatchDev b) {
    extern __shared__ int32_t rows[];
    __shared__ TileShared<BLOCK> sh;
    __shared__ EjfArgs sa;
    __shared__ uint64_t s_red[3][BLOCK / 64];
    __shared__ int32_t s_claim[5];  // pattern, step, tile, all done, tiles of the step
    __shared__ int64_t s_nin;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = b.n_patterns;
    int rot = (int)((blockIdx.x * 7919u) % (unsigned)(N > 0 ? N : 1));
    int idle = 0;
    if (blockIdx.x == 0 && tid < N) {
        for (int q = tid; q < N; q += BLOCK) b.ctl[q].t_pub[0] = (int64_t)wall_clock64();
    }
    // the context's cancel word, read once per workgroup at the start (later
    // only while waiting): a cancelled run leaves before claiming anything
    if (wid == 0 && b.w.cancel) {
        const uint32_t c = ld_sys_u32(b.w.cancel);
        if (lane == 0 && c != 0u) wait_give_up(b.w, WAIT_CANCEL, -1, -1, 0, -1, 0, 0, 0, 0);
    }
    uint64_t hc = 0, hs = 0, hx = 0;
    for (;;) {
        // ---- find a claimable tile (wave 0 scans 64 patterns at a time; the
        // longest-chain preference holds within each group of 64)
        if (wid == 0) {
            int32_t p = -1, s = -1, tile = -1, ntiles = 0;
            bool all_done = false;
            // idle waiting is bounded: progress = some tile finishing somewhere
            uint64_t t_idle = 0;
            uint32_t prog0 = 0;
            int64_t polls = 0;
            for (;;) {
                if (ld_rlx_u32(b.w.abort) != 0u) {  // a wait gave up, or the run was cancelled
                    all_done = true;
                    break;
                }
                bool got = false;
                for (int base = 0; base < N && !got; base += 64) {
                    const int q = (rot + base + lane) % N;
                    bool avail = false;
                    int32_t st = 0, nt = 0, left = 0;
                    if (base + lane < N) {
                        // polling uses relaxed (per-location coherent) loads: an
                        // acquire here would invalidate L1 on every poll
                        st = ld_rlx_i32(&b.ctl[q].stage);
                        const int32_t ns = b.nsteps[q];
                        if (st < ns) {
                            // ntiles[s] is written once (0 -> final) before stage s is
                            // published, so a nonzero value is the final one
                            nt = ld_rlx_i32(&b.ctl[q].ntiles[st]);
                            avail = ld_rlx_i32(&b.ctl[q].claim[st]) < nt;
                            left = ns - st;
                        }
                    }
                    uint64_t m = __ballot(avail);
                    while (m) {
                        // Preference among the claimable patterns still untried:
                        // first those whose home XCD (pattern mod 8) is this
                        // workgroup's (workgroups are dealt to the 8 XCDs
                        // round-robin by index), so a pattern's look-back words
                        // mostly stay in one L2; then the longest chain (most
                        // steps left), so the patterns that set the launch's
                        // length never wait behind short ones; ties in rotated
                        // order.
                        const int32_t pr = left + (((q & 7) == (int)(blockIdx.x & 7)) ? 64 : 0);
                        int32_t mx = ((m >> lane) & 1ull) ? pr : -1;
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
                        const uint64_t top = m & __ballot(((m >> lane) & 1ull) && pr == mx);
                        const int l = __ffsll((long long)top) - 1;
                        m &= ~(1ull << l);
                        const int32_t qq = __shfl(q, l, 64);
                        const int32_t ss = __shfl(st, l, 64);
                        const int32_t ntl = __shfl(nt, l, 64);
                        int32_t t = 0;
                        if (lane == 0) t = atomicAdd(&b.ctl[qq].claim[ss], 1);
                        t = __shfl(t, 0, 64);
                        if (t < ntl) {
                            p = qq;
                            s = ss;
                            tile = t;
                            ntiles = ntl;
                            got = true;
                            break;
                        }
                    }
                }
                if (got) break;
                if (ld_rlx_i32(b.finished) >= N) {
                    all_done = true;
                    break;
                }
                polls++;
                const uint32_t prog = ld_rlx_u32(b.tiles_done);
                const uint64_t now = wall_clock64();
                if (t_idle == 0 || prog != prog0) {
                    t_idle = now;
                    prog0 = prog;
                } else if (now - t_idle > b.w.limit) {
                    // nothing finished anywhere for the whole limit: name the
                    // first unfinished pattern and leave
                    if (lane == 0) {
                        int32_t q = 0, st = -1;
                        for (; q < N; q++) {
                            st = ld_rlx_i32(&b.ctl[q].stage);
                            if (st < b.nsteps[q]) break;
                        }
                        int32_t nt = 0, cl = 0, dn = 0;
                        if (q < N) {
                            nt = ld_rlx_i32(&b.ctl[q].ntiles[st]);
                            cl = ld_rlx_i32(&b.ctl[q].claim[st]);
                            dn = ld_rlx_i32(&b.ctl[q].done[st]);
                        }
                        wait_give_up(b.w, WAIT_IDLE, q < N ? q : -1, st, nt, -1, polls, now - t_idle, cl, dn);
                    }
                    all_done = true;
                    break;
                }
                if ((polls & 31) == 0 && b.w.cancel && ld_sys_u32(b.w.cancel) != 0u) {
                    if (lane == 0) wait_give_up(b.w, WAIT_CANCEL, -1, -1, 0, -1, polls, now - t_idle, 0, 0);
                    all_done = true;
                    break;
                }
                // idle: back off exponentially so polling does not flood the memory system
                for (int i = 0; i < idle; i++) __builtin_amdgcn_s_sleep(16);
                idle = idle < b.max_backoff ? 2 * idle + 1 : idle;
            }
            idle = 0;
            if (lane == 0) {
                s_claim[0] = p;
                s_claim[1] = s;
                s_claim[2] = tile;
                s_claim[3] = all_done ? 1 : 0;
                s_claim[4] = ntiles;
            }
        }
        __syncthreads();
        const int32_t p = s_claim[0], s = s_claim[1];
        const int64_t tile = s_claim[2];
        const bool all_done = s_claim[3] != 0;
        const int64_t n_tiles = s_claim[4];
        __syncthreads();  // s_claim is rewritten by the next scan
        if (all_done) break;
        rot = (p + 1) % N;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // ---- stage the step's arguments in LDS
        {
            const int32_t* src = (const int32_t*)&b.args[b.first[p] + s];
            int32_t* dst = (int32_t*)&sa;
            for (int i = tid; i < (int)(sizeof(EjfArgs) / 4); i += BLOCK) dst[i] = src[i];
            if (tid == 0) s_nin = b.ctl[p].n_in[s];  // written before the step was published
        }
        __syncthreads();
        const int64_t n_in = s_nin;
        ejf_tile<BLOCK, NV, false, true>(sa, nullptr, tile, n_in, n_tiles, sh, rows, hc, hs, hx);
        if (sa.mode == EJF_HASH) {
            hash_flush<BLOCK>(sa.hash_acc, hc, hs, hx, s_red);
            hc = hs = hx = 0;
        }
        // ---- completion: the last tile of a step publishes the next one
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();  // every wave's stores are released before the count
        if (tid == 0) {
            const int32_t d = atomicAdd(&b.ctl[p].done[s], 1);
            __hip_atomic_fetch_add(b.tiles_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (d == n_tiles - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                BatchCtl& c = b.ctl[p];
                const int32_t ns = b.nsteps[p];
                const int64_t n_out = (sa.mode == EJF_HASH) ? 0 : __hip_atomic_load(sa.n_out, __ATOMIC_RELAXED,
                                                                                       __HIP_MEMORY_SCOPE_AGENT);
                bool next = false;
                if (s + 1 < ns && n_out > 0) {
                    // publish step s + 1: cut its output table (rows = the exact
                    // candidate bound) and its look-back words from the heap
                    EjfArgs& nx = b.args[b.first[p] + s + 1];
                    const int64_t nn = clamp_rows(n_out, sa.out_cap);
                    int64_t rows_out = 0;
                    if (nx.mode == EJF_WRITE)
                        rows_out = nx.st.motif >= 0
                                       ? (int64_t)__hip_atomic_load((unsigned long long*)&c.cand[s + 1],
                                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                       : nn;
                    if (b.row_limit > 0 && rows_out > b.row_limit) rows_out = b.row_limit;
                    const int c_out = nx.st.c_in + (nx.st.motif >= 0 ? nx.st.n_new : 0);
                    const int64_t elems = (rows_out * c_out + 63) & ~(int64_t)63;
                    const int64_t ntl = (nn + BLOCK - 1) / BLOCK;
                    const int64_t words = ntl + 2;
                    const int64_t off = (int64_t)atomicAdd(b.heap_top, (unsigned long long)elems);
                    const int64_t woff = (int64_t)atomicAdd(b.words_top, (unsigned long long)words);
                    if (off + elems <= b.heap_cap && woff + words <= b.words_cap) {
                        nx.in = sa.out;
                        nx.in_stride = sa.out_stride;
                        nx.in_cap = sa.out_cap;
                        nx.out = b.heap + off;
                        nx.out_stride = rows_out > 0 ? rows_out : 1;
                        nx.out_cap = rows_out;
                        nx.status = b.words + woff;
                        c.n_in[s + 1] = nn;
                        c.t_pub[s + 1] = (int64_t)wall_clock64();
                        __hip_atomic_store(&c.ntiles[s + 1], (int32_t)ntl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                        st_rel_i32(&c.stage, s + 1);
                        next = true;
                    } else {
                        b.heap_fail[p] = 1;
                    }
                } else if (s + 1 == ns && sa.mode == EJF_WRITE && n_out > 0 && b.jobs) {
                    // the final table goes to the sort, with 2 * rows index scratch
                    SortJob& j = b.jobs[p];
                    const int64_t nn = clamp_rows(n_out, sa.out_cap);
                    const int64_t elems = (2 * nn + 63) & ~(int64_t)63;
                    const int64_t off = (int64_t)atomicAdd(b.heap_top, (unsigned long long)elems);
                    if (off + elems <= b.heap_cap) {
                        j.in = sa.out;
                        j.in_stride = sa.out_stride;
                        j.in_cap = sa.out_cap;
                        j.scratch_idx = (uint32_t*)(b.heap + off);
                    } else {
                        b.heap_fail[p] = 1;
                    }
                }
                if (!next) {
                    // last step, nothing left or no room: the remaining steps produce 0 rows
                    for (int q = s + 1; q < ns; q++) *b.args[b.first[p] + q].n_out = 0;
                    c.t_pub[ns] = (int64_t)wall_clock64();
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    st_rel_i32(&c.stage, ns);
                    atomicAdd(b.finished, 1);
                }
            }
        }
        __syncthreads();
    }
}

int batch_block_for(int max_cols, int requested) {
    // the LDS row tile stays within ~32 KB
    const int cap = max_cols <= 31 ? 256 : (max_cols <= 63 ? 128 : 64);
    int blk = requested > 0 ? requested : cap;
    return blk > cap ? cap : blk;
}

int batch_grid_for(int block, int max_cols, int requested) {
    const size_t lds = sizeof(int32_t) * (size_t)block * row_stride(max_cols);
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (block) {
        case 64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<64, kNarrowNew>, 64, lds); break;
        case 128: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<128, kNarrowNew>, 128, lds); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<256, kNarrowNew>, 256, lds); break;
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    const int resident = per_cu * cus;
    // one 256-thread workgroup per CU (the same threads per CU for the
    // narrower blocks): measured best on 256 CUs, 0.84 ms against 0.90 ms at
    // 1.5 per CU and 1.05 ms at 2 (more workgroups mean more scheduler polls,
    // claims and per-tile fences contending), 0.90 ms at 0.75 per CU
    const int want = requested > 0 ? requested : (block >= 256 ? cus : (block == 128 ? 2 * cus : 4 * cus));
    return want < resident ? want : resident;
}

hipError_t launch_batch(const BatchDev& b, int block, int max_cols, bool wide, int grid, hipStream_t s) {
    const size_t lds = sizeof(int32_t) * (size_t)block * row_stride(max_cols);
    if (wide) {
        switch (block) {
            case 64: hipLaunchKernelGGL((batch_kernel<64, kMaxMotif>), dim3(grid), dim3(64), lds, s, b); break;
            case 128: hipLaunchKernelGGL((batch_kernel<128, kMaxMotif>), dim3(grid), dim3(128), lds, s, b); break;
            default: hipLaunchKernelGGL((batch_kernel<256, kMaxMotif>), dim3(grid), dim3(256), lds, s, b); break;
        }
    } else {
        switch (block) {
            case 64: hipLaunchKernelGGL((batch_kernel<64, kNarrowNew>), dim3(grid), dim3(64), lds, s, b); break;
            case 128: hipLaunchKernelGGL((batch_kernel<128, kNarrowNew>), dim3(grid), dim3(128), lds, s, b); break;
            default: hipLaunchKernelGGL((batch_kernel<256, kNarrowNew>), dim3(grid), dim3(256), lds, s, b); break;
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonicalization: per-root-segment lexicographic sort
// ---------------------------------------------------------------------------
//
// The join steps keep their input order, and the first table is the identity
// (one row per root vertex, ascending), so a final table is already grouped
// by the root column in ascending order.  Canonicalization therefore sorts
// each root segment independently: in LDS when it fits (two tiers of LDS
// size), else with a global-memory bitonic sort of row indices.  Columns are
// permuted to pattern-vertex order on the way and the output is row-major.

__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* a, int64_t n, int32_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

constexpr int kSortBlock = 256;

__device__ __forceinline__ bool lds_row_less(const uint64_t* rows, int wp, uint32_t x, uint32_t y) {
    const uint64_t* a = rows + (size_t)x * wp;
    const uint64_t* b = rows + (size_t)y * wp;
    for (int w = 0; w < wp; w++) {
        const uint64_t p = a[w], q = b[w];
        if (p != q) return p < q;
    }
    return false;
}

constexpr uint16_t kSent16 = 0xFFFFu;

// The run of value v in the ascending a[0, n), found by one full wave: lanes
// 0-31 look for the first element >= v, lanes 32-63 for the first > v.  Each
// round a half probes 32 evenly spaced positions of the interval that still
// holds its answer, so both ends take ~log32(n) dependent loads together.
__device__ void wave_equal_range(const int32_t* a, int64_t n, int32_t v, int lane, int64_t* first, int64_t* end) {
    const int half = lane >> 5, hl = lane & 31;
    const int32_t t = half ? v + 1 : v;  // v < INT32_MAX: vertex ids
    int64_t lo = 0, hi = n;              // this half's answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t step = (hi - lo + 31) / 32;
        int64_t p = lo + (int64_t)(hl + 1) * step - 1;
        if (p > hi - 1) p = hi - 1;
        const uint32_t m = (uint32_t)(__ballot(a[p] >= t) >> (32 * half));
        if (m == 0) {
            lo = hi;
            break;
        }
        const int f = __ffs((int)m) - 1;
        int64_t pf = lo + (int64_t)(f + 1) * step - 1;
        if (pf > hi - 1) pf = hi - 1;
        lo = f == 0 ? lo : lo + (int64_t)f * step;  // one past the probe of lane f - 1
        hi = pf;
    }
    if (hl == 0) {
        if (half) *end = lo;
        else *first = lo;
    }
}

// Sort the n packed rows staged in LDS with a bitonic network over 16-bit
// row indices; idx[0, n) receives the order.  Called by the whole workgroup.
// The pairs t of one wave (64 consecutive t, for each multiple of the block
// size) are (lo, lo + stride) with lo = t + (t & ~(stride - 1)): for stride <=
// 64 they lie inside the wave's own 128-element chunk, so a run of such stages
// needs no workgroup barrier, only a wavefront-scope fence that orders one
// stage's LDS stores before the next stage's loads across the wave's lanes;
// a stage with a longer stride, or the first stage after one, waits for all.
__device__ void lds_bitonic(const uint64_t* rows, uint16_t* idx, int n, int wp) {
    const int tid = threadIdx.x, nt = (int)blockDim.x;
    int P = 1;
    while (P < n) P <<= 1;
    for (int i = tid; i < P; i += nt) idx[i] = i < n ? (uint16_t)i : kSent16;
    __syncthreads();
    int prev = 0;  // stride of the previous stage (0: the fill, followed by a barrier)
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (prev != 0) {
                if (stride > 64 || prev > 64) {
                    __syncthreads();
                } else {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            prev = stride;
            for (int t = tid; t < (P >> 1); t += nt) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint16_t ia = idx[lo], ib = idx[hi];
                bool gt;
                if (ia == kSent16) gt = (ib != kSent16);
                else if (ib == kSent16) gt = false;
                else gt = lds_row_less(rows, wp, ib, ia);
                if (gt == asc) {
                    idx[lo] = ib;
                    idx[hi] = ia;
                }
            }
        }
    }
    __syncthreads();
}

// Stage rows [r0, r0 + n) of a final table into LDS as packed rows
// (columns 1..k-1 in pattern-vertex order).  Work is dealt by element,
// column-major so neighbouring lanes read neighbouring rows of one column;
// each thread issues eight independent loads before OR-ing the values into
// the zeroed words, so a row's columns are fetched in parallel, not in turn.
// A thread's (column, row) advances by a fixed step: no division per element.
__device__ __forceinline__ void lds_stage_rows(const SortJob& job, int64_t r0, int n, uint64_t* rows) {
    const int k = job.k, wp = job.wp, bits = job.bits, cpw = job.cpw;
    const int nt = (int)blockDim.x;
    for (int i = threadIdx.x; i < n * wp; i += nt) rows[i] = 0;
    __syncthreads();
    const int total = n * (k - 1);
    const int dj = nt / n, dr = nt - dj * n;  // element step nt = dj columns + dr rows
    int j = 1 + (int)threadIdx.x / n, r = (int)threadIdx.x % n;
    for (int e0 = threadIdx.x; e0 < total; e0 += 8 * nt) {
        uint32_t v[8];
        int jj[8], rr[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            jj[u] = j;
            rr[u] = r;
            v[u] = 0;
            if (e0 + u * nt < total) v[u] = (uint32_t)job.in[(int64_t)job.perm[j] * job.in_stride + r0 + r];
            j += dj;
            r += dr;
            if (r >= n) {
                r -= n;
                j++;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            if (e0 + u * nt < total) {
                const int q = (jj[u] - 1) / cpw, c = (jj[u] - 1) - q * cpw;
                atomicOr((unsigned long long*)&rows[(size_t)rr[u] * wp + q],
                         (unsigned long long)v[u] << ((cpw - 1 - c) * bits));
            }
        }
    }
    __syncthreads();
}

// Write rows idx[0, nw) of the packed tile as row-major int32 rows of k
// columns at dst (column 0 = root): one row per thread, its words read once
// and unpacked in registers.
__device__ __forceinline__ void lds_write_rows(const uint64_t* rows, const uint16_t* idx, const SortJob& job,
                                               int nw, int32_t root, int32_t* dst) {
    const int k = job.k, wp = job.wp, bits = job.bits, cpw = job.cpw;
    const uint64_t mask = (1ull << bits) - 1;
    for (int r = threadIdx.x; r < nw; r += (int)blockDim.x) {
        const uint64_t* src = rows + (size_t)idx[r] * wp;
        int32_t* o = dst + (int64_t)r * k;
        o[0] = root;
        int j = 1;
        for (int w = 0; w < wp && j < k; w++) {
            const uint64_t word = src[w];
            for (int c = 0; c < cpw && j < k; c++, j++) o[j] = (int32_t)((word >> ((cpw - 1 - c) * bits)) & mask);
        }
    }
}

__device__ __forceinline__ void push_segment(const SortLaunch& L, int32_t item, int64_t seg0, int64_t len) {
    const int32_t q = atomicAdd(L.spill_n, 1);
    SegRef r;
    r.item = item;
    r.pad_ = 0;
    r.seg0 = seg0;
    r.len = len;
    L.spill[q] = r;
}

// Compare rows x and y of a segment straight from the table's columns.
__device__ __forceinline__ int glb_row_cmp(const SortJob& a, int64_t seg0, uint32_t x, uint32_t y) {
    for (int j = 1; j < a.k; j++) {
        const int32_t* c = a.in + (int64_t)a.perm[j] * a.in_stride + seg0;
        const int32_t p = c[x], q = c[y];
        if (p != q) return p < q ? -1 : 1;
    }
    return 0;
}

// Copy the rows [seg0, seg0 + len) of a final table to the row-major output
// in pattern-vertex order (rows below out_rows only), checking on the way
// that they increase strictly, in chunks staged in LDS: each column of a
// chunk is read coalesced, the rows are compared with their predecessors
// (the previous chunk's last row is kept), and the chunk is written
// row-major, coalesced.  Stops at the first chunk out of order and returns
// false (what was written is overwritten by the sort); true when the whole
// segment was in order.  tile: at least k * (CH + 1) + k int32 of LDS with
// CH = chunk rows.  Called by the whole workgroup.
__device__ bool copy_if_sorted(const SortJob& job, int64_t seg0, int64_t len, int64_t out_rows, int32_t* tile,
                               int lds_words) {
    const int k = job.k, nt = (int)blockDim.x, tid = threadIdx.x;
    int ch = (lds_words - k) / k - 1;  // chunk rows; stride ch + 1 is odd or at least not a bank multiple
    if (ch > 1024) ch = 1024;
    if (ch < 1) return false;
    const int cs = ch + 1;
    int32_t* prev = tile + (size_t)k * cs;
    for (int64_t r0 = 0; r0 < len; r0 += ch) {
        const int n = (int)((len - r0 < ch) ? (len - r0) : ch);
        // stage: element e = j * n + r, (column, row) stepped without a division
        {
            const int dj = nt / n, dr = nt - dj * n;
            int j = tid / n, r = tid - j * n;
            for (int e = tid; e < n * k; e += nt) {
                tile[j * cs + r] = job.in[(int64_t)job.perm[j] * job.in_stride + seg0 + r0 + r];
                j += dj;
                r += dr;
                if (r >= n) {
                    r -= n;
                    j++;
                }
            }
        }
        __syncthreads();
        int bad = 0;
        for (int r = tid; r < n; r += nt) {
            if (r0 == 0 && r == 0) continue;
            int c = 0;
            for (int j = 1; j < k && c == 0; j++) {
                const int32_t a = r > 0 ? tile[j * cs + r - 1] : prev[j], b = tile[j * cs + r];
                c = a < b ? -1 : (a > b ? 1 : 0);
            }
            bad |= c >= 0;
        }
        if (__syncthreads_or(bad)) return false;
        const int64_t left = out_rows - (seg0 + r0);
        const int nw = left <= 0 ? 0 : (left < n ? (int)left : n);
        {
            int32_t* dst = job.out + (seg0 + r0) * k;
            const int dr = nt / k, dj = nt - dr * k;
            int r = tid / k, j = tid - r * k;
            for (int e = tid; e < nw * k; e += nt) {
                dst[e] = tile[j * cs + r];
                r += dr;
                j += dj;
                if (j >= k) {
                    j -= k;
                    r++;
                }
            }
        }
        if (job.out_cost)
            for (int r = tid; r < nw; r += nt) job.out_cost[seg0 + r0 + r] = job.in_cost[seg0 + r0 + r];
        if (tid < k) prev[tid] = tile[tid * cs + n - 1];
        __syncthreads();
    }
    return true;
}

// LDS tiers: one workgroup per root segment.  Without an input list the items
// are every (job, root vertex) pair and the segment is found by search;
// segments larger than this tier's LDS tile are passed on.
__global__ __launch_bounds__(1024) void sort_lds_kernel(const SortLaunch L) {
    extern __shared__ uint64_t lds[];
    __shared__ SortJob job;
    __shared__ int64_t s_seg[2];
    const int tid = threadIdx.x;
    if (L.abort && *L.abort) return;  // set by an earlier launch of the run: stable here
    const int64_t n_items = L.list ? (int64_t)*L.list_n : (int64_t)L.n_jobs * L.n_vertices;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int32_t item = L.list ? L.list[it].item : (int32_t)it;
        // after the streaming pass: only the segments it found out of order
        if (L.todo && L.todo[item] != L.todo_epoch) continue;
        const int64_t jb = item / L.n_vertices;
        {
            const int32_t* src = L.jobs ? (const int32_t*)&L.jobs[jb] : (const int32_t*)&L.one;
            int32_t* dst = (int32_t*)&job;
            for (int i = tid; i < (int)(sizeof(SortJob) / 4); i += (int)blockDim.x) dst[i] = src[i];
        }
        __syncthreads();
        if (L.list) {
            if (tid == 0) {
                s_seg[0] = L.list[it].seg0;
                s_seg[1] = L.list[it].len;
            }
        } else if (tid < 64) {
            const int32_t v = L.v_begin + (int32_t)(item - jb * L.n_vertices);
            const int64_t n = clamp_rows(*job.n_in, job.in_cap);
            wave_equal_range(job.in, n, v, tid, &s_seg[0], &s_seg[1]);
        }
        __syncthreads();
        const int64_t seg0 = s_seg[0], len = L.list ? s_seg[1] : s_seg[1] - s_seg[0];
        const int k = job.k, wp = job.wp;
        const int64_t out_rows = job.out_rows;
        const int cap_rows = lds_rows_of(L.lds_bytes, wp);
        __syncthreads();  // every lane has read job and s_seg: the next item may overwrite them
        if (len == 0 || seg0 >= out_rows) continue;
        // a segment the joins left in order (paths placed in label order, and
        // every join that extends rows with candidates in ascending order)
        // needs no sort: copied out in one coalesced pass while it is checked
        if (!L.list && copy_if_sorted(job, seg0, len, out_rows, (int32_t*)lds, L.lds_bytes / 4)) continue;
        if (len > cap_rows) {
            if (tid == 0) push_segment(L, item, seg0, len);
            continue;
        }
        const int n = (int)len;
        uint64_t* rows = lds;
        uint16_t* idx = (uint16_t*)(lds + (size_t)cap_rows * wp);
        const int32_t root = job.in[(int64_t)job.perm[0] * job.in_stride + seg0];
        lds_stage_rows(job, seg0, n, rows);
        int uns = 0;
        for (int r = tid + 1; r < n; r += (int)blockDim.x) uns |= !lds_row_less(rows, wp, r - 1, r);
        if (__syncthreads_or(uns)) {
            lds_bitonic(rows, idx, n, wp);
            for (int r = tid + 1; r < n; r += (int)blockDim.x)
                if (!lds_row_less(rows, wp, idx[r - 1], idx[r])) atomicAdd(L.dup_count, 1);
        } else {
            // already in order (strictly, so free of duplicates)
            for (int r = tid; r < n; r += (int)blockDim.x) idx[r] = (uint16_t)r;
            __syncthreads();
        }
        const int64_t nw = (seg0 + n <= out_rows) ? n : (out_rows - seg0);
        lds_write_rows(rows, idx, job, (int)nw, root, job.out + seg0 * k);
        if (job.out_cost)
            for (int64_t r = tid; r < nw; r += (int)blockDim.x) job.out_cost[seg0 + r] = job.in_cost[seg0 + idx[r]];
        __syncthreads();
    }
}

// Rows per tile of the streaming pass for k columns (about 16 KB of LDS).
__host__ __device__ __forceinline__ int stream_tile_rows(int k) { return k <= 16 ? 256 : (k <= 32 ? 128 : 64); }

// The streaming pass over one job's table: tiles of T rows staged column by
// column (pattern order) in LDS, each row compared with the one before it
// (the tile's first with the previous tile's last, read again), rows written
// row-major with coalesced stores.  Neighbours in one root segment that are
// not strictly increasing flag the segment (its bit, set once) or, when
// equal, count as a duplicate.
__global__ __launch_bounds__(256) void sort_stream_kernel(const SortLaunch L, uint32_t* unsorted, int32_t* n_unsorted) {
    extern __shared__ int32_t tile[];
    __shared__ SortJob job;
    const int tid = threadIdx.x, nt = (int)blockDim.x;
    if (L.abort && *L.abort) return;
    {
        const int32_t* src = L.jobs ? (const int32_t*)&L.jobs[0] : (const int32_t*)&L.one;
        int32_t* dst = (int32_t*)&job;
        for (int i = tid; i < (int)(sizeof(SortJob) / 4); i += nt) dst[i] = src[i];
    }
    __syncthreads();
    const int k = job.k;
    const int T = stream_tile_rows(k), cs = T + 1;
    int32_t* prev = tile + (size_t)k * cs;
    const int64_t n = clamp_rows(*job.n_in, job.in_cap);
    const int64_t out_rows = job.out_rows;
    const int64_t stride = job.in_stride;
    const int shiftT = T == 256 ? 8 : (T == 128 ? 7 : 6);
    for (int64_t r0 = (int64_t)blockIdx.x * T; r0 < n; r0 += (int64_t)gridDim.x * T) {
        const int m = (int)((n - r0 < T) ? (n - r0) : T);
        for (int e = tid; e < k * T; e += nt) {
            const int j = e >> shiftT, r = e & (T - 1);
            if (r < m) tile[j * cs + r] = job.in[(int64_t)job.perm[j] * stride + r0 + r];
        }
        if (r0 > 0 && tid < k) prev[tid] = job.in[(int64_t)job.perm[tid] * stride + r0 - 1];
        __syncthreads();
        for (int r = tid; r < m; r += nt) {
            if (r0 + r == 0) continue;
            const int32_t root = tile[r];
            if ((r > 0 ? tile[r - 1] : prev[0]) != root) continue;  // first row of its segment
            int c = 0;
            for (int j = 1; j < k && c == 0; j++) {
                const int32_t a = r > 0 ? tile[j * cs + r - 1] : prev[j], b = tile[j * cs + r];
                c = a < b ? -1 : (a > b ? 1 : 0);
            }
            if (c == 0) {
                atomicAdd(L.dup_count, 1);
            } else if (c > 0) {
                // the segment's word takes this pass's epoch; the first to set it counts it
                const int32_t item = root - L.v_begin;
                const uint32_t ep = L.todo_epoch;
                if (__hip_atomic_load(&unsorted[item], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep)
                    if (atomicExch(&unsorted[item], ep) != ep) atomicAdd(n_unsorted, 1);
            }
        }
        const int64_t left = out_rows - r0;
        const int nw = left <= 0 ? 0 : (left < m ? (int)left : m);
        {
            int32_t* dst = job.out + r0 * k;
            const int dr = nt / k, dj = nt - dr * k;
            int r = tid / k, j = tid - r * k;
            for (int e = tid; e < nw * k; e += nt) {
                dst[e] = tile[j * cs + r];
                r += dr;
                j += dj;
                if (j >= k) {
                    j -= k;
                    r++;
                }
            }
        }
        if (job.out_cost)
            for (int r = tid; r < nw; r += nt) job.out_cost[r0 + r] = job.in_cost[r0 + r];
        __syncthreads();
    }
}

hipError_t launch_sort_stream(const SortLaunch& a, uint32_t* unsorted, int32_t* n_unsorted, int64_t in_cap_rows, int k,
                              hipStream_t s) {
    const int T = stream_tile_rows(k);
    const size_t lds = sizeof(int32_t) * ((size_t)k * (T + 1) + (size_t)k);
    const int64_t tiles = (std::max<int64_t>(in_cap_rows, 1) + T - 1) / T;
    const int grid = (int)std::min<int64_t>(tiles, 4096);
    hipLaunchKernelGGL(sort_stream_kernel, dim3(grid), dim3(256), lds, s, a, unsorted, n_unsorted);
    return hipGetLastError();
}

// ---- merge tier, for segments larger than the largest LDS tile --------------
//
// The segment is cut into chunks of the LDS tile's row count; each chunk is
// sorted in LDS into a run of row indices, then runs are merged pairwise,
// one launch per pass: an element's place in the merged run is its place in
// its own run plus its rank in the partner run (binary search comparing rows
// in the table).  Indices ping-pong between the two halves of the job's
// index scratch at 2 * seg0; a last launch writes the rows.  Every launch
// spreads each segment's work over all workgroups, starting at a different
// workgroup per segment.


__device__ __forceinline__ int ceil_log2_i64(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) r++;
    return r;
}

// first unit of segment i that workgroup b handles when units are dealt round-robin
__device__ __forceinline__ int64_t first_unit(int64_t i) {
    const int64_t G = gridDim.x;
    return ((int64_t)blockIdx.x + G - (i % G)) % G;
}

__global__ __launch_bounds__(1024) void sort_chunk_kernel(const SortLaunch L) {
    extern __shared__ uint64_t lds[];
    const int tid = threadIdx.x;
    if (L.abort && *L.abort) return;  // set by an earlier launch of the run: stable here
    const int64_t n_list = *L.list_n;
    for (int64_t i = 0; i < n_list; i++) {
        const SegRef ref = L.list[i];
        const SortJob& job = L.jobs[ref.item / L.n_vertices];
        const int wp = job.wp;
        const int R = lds_rows_of(L.lds_bytes, wp);
        const int64_t nch = (ref.len + R - 1) / R;
        if (blockIdx.x == 0 && tid == 0) atomicMax(L.max_chunks, (int32_t)(nch < INT32_MAX ? nch : INT32_MAX));
        uint32_t* run = job.scratch_idx + 2 * ref.seg0;
        uint64_t* rows = lds;
        uint16_t* idx = (uint16_t*)(lds + (size_t)R * wp);
        for (int64_t c = first_unit(i); c < nch; c += gridDim.x) {
            const int64_t r0 = c * R;
            const int n = (int)((ref.len - r0 < R) ? (ref.len - r0) : R);
            lds_stage_rows(job, ref.seg0 + r0, n, rows);
            int uns = 0;
            for (int r = tid + 1; r < n; r += (int)blockDim.x) uns |= !lds_row_less(rows, wp, r - 1, r);
            if (__syncthreads_or(uns)) {
                lds_bitonic(rows, idx, n, wp);
            } else {
                for (int r = tid; r < n; r += (int)blockDim.x) idx[r] = (uint16_t)r;
                __syncthreads();
            }
            for (int r = tid; r < n; r += (int)blockDim.x) run[r0 + r] = (uint32_t)(r0 + idx[r]);
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(kSortBlock) void sort_merge_kernel(const SortLaunch L) {
    if (L.abort && *L.abort) return;  // set by an earlier launch of the run: stable here
    const int p = L.pass;
    if (((int64_t)1 << p) >= (int64_t)*L.max_chunks) return;  // every segment is one run already
    const int tid = threadIdx.x;
    const int64_t n_list = *L.list_n;
    const int64_t G = gridDim.x;
    for (int64_t i = 0; i < n_list; i++) {
        const SegRef ref = L.list[i];
        const SortJob& job = L.jobs[ref.item / L.n_vertices];
        const int R = lds_rows_of(L.lds_bytes, job.wp);
        const int64_t len = ref.len;
        const int64_t nch = (len + R - 1) / R;
        if (((int64_t)1 << p) >= nch) continue;  // this segment needs fewer passes
        const uint32_t* in = job.scratch_idx + 2 * ref.seg0 + ((p & 1) ? len : 0);
        uint32_t* out = job.scratch_idx + 2 * ref.seg0 + ((p & 1) ? 0 : len);
        const int64_t w = (int64_t)R << p;
        for (int64_t e = first_unit(i) * kSortBlock + tid; e < len; e += G * kSortBlock) {
            const uint32_t x = in[e];
            const int64_t r = e / w, rs = r * w, ps = (r ^ 1) * w;
            if (ps >= len) {  // no partner run in this pass
                out[e] = x;
                continue;
            }
            const int64_t pe = (ps + w < len) ? ps + w : len;
            const bool left = (r & 1) == 0;
            int64_t lo = ps, hi = pe;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int c = glb_row_cmp(job, ref.seg0, in[mid], x);
                if (left ? (c < 0) : (c <= 0)) lo = mid + 1; else hi = mid;
            }
            out[(rs < ps ? rs : ps) + (e - rs) + (lo - ps)] = x;
        }
    }
}

__global__ __launch_bounds__(kSortBlock) void sort_gather_kernel(const SortLaunch L) {
    if (L.abort && *L.abort) return;  // set by an earlier launch of the run: stable here
    const int tid = threadIdx.x;
    const int64_t n_list = *L.list_n;
    const int64_t G = gridDim.x;
    for (int64_t i = 0; i < n_list; i++) {
        const SegRef ref = L.list[i];
        const SortJob& job = L.jobs[ref.item / L.n_vertices];
        const int k = job.k;
        const int R = lds_rows_of(L.lds_bytes, job.wp);
        const int64_t len = ref.len;
        const int np = ceil_log2_i64((len + R - 1) / R);
        const uint32_t* idx = job.scratch_idx + 2 * ref.seg0 + ((np & 1) ? len : 0);
        for (int64_t e = first_unit(i) * kSortBlock + tid; e < len; e += G * kSortBlock)
            if (e > 0 && glb_row_cmp(job, ref.seg0, idx[e - 1], idx[e]) >= 0) atomicAdd(L.dup_count, 1);
        const int64_t nw = (ref.seg0 + len <= job.out_rows) ? len : (job.out_rows - ref.seg0);
        const int64_t total = nw * k;
        int32_t* dst = job.out + ref.seg0 * k;
        for (int64_t e = first_unit(i) * kSortBlock + tid; e < total; e += G * kSortBlock) {
            const int64_t r = e / k;
            const int j = (int)(e - r * k);
            dst[e] = job.in[(int64_t)job.perm[j] * job.in_stride + ref.seg0 + idx[r]];
        }
        if (job.out_cost)
            for (int64_t r = first_unit(i) * kSortBlock + tid; r < nw; r += G * kSortBlock)
                job.out_cost[ref.seg0 + r] = job.in_cost[ref.seg0 + idx[r]];
    }
}

// ---------------------------------------------------------------------------
// top-k by (cost, position) over a sorted table with a cost per row
// ---------------------------------------------------------------------------
//
// Phases 0..7 select the threshold cost T digit by digit (8 bits, most
// significant first) among the rows still in the candidate class; phases
// 8..11 select, among the rows costing exactly T, the position P of the
// (k - #rows below T)-th one.  The winners are then the rows with cost < T
// and those with cost == T at a position <= P: exactly k rows.

__global__ void topk_init_kernel(TopkCtl* ctl, int64_t k) {
    const int t = threadIdx.x;
    if (t == 0) {
        ctl->prefix = 0;
        ctl->k_rem = k;
        ctl->n_less = 0;
        ctl->n_out = 0;
        ctl->t_cost = 0;
    }
    for (int i = t; i < 256; i += blockDim.x) ctl->hist[i] = 0;
}

__device__ __forceinline__ int topk_shift(int phase) { return phase < 8 ? 56 - 8 * phase : 24 - 8 * (phase - 8); }

__global__ __launch_bounds__(256) void topk_hist_kernel(const uint64_t* cost, int64_t n, TopkCtl* ctl, int phase) {
    __shared__ unsigned int h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int shift = topk_shift(phase);
    const unsigned long long prefix = ctl->prefix;
    const unsigned long long t_cost = ctl->t_cost;
    const bool by_cost = phase < 8;
    const unsigned long long above = (by_cost ? (phase == 0 ? 0ull : ~0ull << (shift + 8))
                                              : (phase == 8 ? 0ull : ~0ull << (shift + 8)));
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long c = cost[i];
        unsigned long long key;
        if (by_cost) {
            key = c;
        } else {
            if (c != t_cost) continue;
            key = (unsigned long long)i;
        }
        if (((key ^ prefix) & above) != 0) continue;
        atomicAdd(&h[(key >> shift) & 255ull], 1u);
    }
    __syncthreads();
    if (h[tid]) atomicAdd(&ctl->hist[tid], h[tid]);
}

__global__ void topk_pick_kernel(TopkCtl* ctl, int phase) {
    if (threadIdx.x == 0) {
        const long long k = ctl->k_rem;
        long long cum = 0;
        int d = 0;
        for (; d < 255; d++) {
            if (cum + (long long)ctl->hist[d] >= k) break;
            cum += ctl->hist[d];
        }
        ctl->k_rem = k - cum;
        ctl->prefix |= (unsigned long long)d << topk_shift(phase);
        if (phase < 8) ctl->n_less += cum;
        if (phase == 7) {
            ctl->t_cost = ctl->prefix;
            ctl->prefix = 0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x) ctl->hist[i] = 0;
}

__global__ __launch_bounds__(256) void topk_gather_kernel(const uint64_t* cost, int64_t n, TopkCtl* ctl,
                                                          uint64_t* sel_cost, uint32_t* sel_pos) {
    const unsigned long long t = ctl->t_cost, p = ctl->prefix;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long c = cost[i];
        if (c < t || (c == t && (unsigned long long)i <= p)) {
            const unsigned long long j = atomicAdd(&ctl->n_out, 1ull);
            sel_cost[j] = c;
            sel_pos[j] = (uint32_t)i;
        }
    }
}

// One workgroup: bitonic sort of the k winners by (cost, position) in LDS,
// then their rows and costs are written in that order.
__global__ __launch_bounds__(1024) void topk_sort_kernel(const uint64_t* sel_cost, const uint32_t* sel_pos, int32_t k,
                                                         const int32_t* table, int32_t width, int32_t* out_rows,
                                                         uint64_t* out_cost) {
    extern __shared__ uint64_t sm[];
    int P = 1;
    while (P < k) P <<= 1;
    uint64_t* kc = sm;
    uint32_t* kp = (uint32_t*)(sm + P);
    const int tid = threadIdx.x;
    for (int i = tid; i < P; i += blockDim.x) {
        kc[i] = i < k ? sel_cost[i] : ~0ull;
        kp[i] = i < k ? sel_pos[i] : 0xFFFFFFFFu;
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < (P >> 1); t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t ca = kc[lo], cb = kc[hi];
                const uint32_t pa = kp[lo], pb = kp[hi];
                const bool gt = ca > cb || (ca == cb && pa > pb);
                if (gt == asc) {
                    kc[lo] = cb;
                    kc[hi] = ca;
                    kp[lo] = pb;
                    kp[hi] = pa;
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += blockDim.x) out_cost[i] = kc[i];
    for (int64_t e = tid; e < (int64_t)k * width; e += blockDim.x) {
        const int64_t r = e / width;
        const int j = (int)(e - r * width);
        out_rows[e] = table[(int64_t)kp[r] * width + j];
    }
}

hipError_t launch_topk(const uint64_t* cost, int64_t n, int64_t k, TopkCtl* ctl, uint64_t* sel_cost,
                       uint32_t* sel_pos, const int32_t* table, int32_t width, int32_t* out_rows,
                       uint64_t* out_cost, hipStream_t s) {
    if (k <= 0 || k > kTopkMax || k > n) return hipErrorInvalidValue;
    static const bool lds_ok = [] {
        const bool ok = hipFuncSetAttribute((const void*)topk_sort_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            12 * kTopkMax) == hipSuccess;
        if (!ok) (void)hipGetLastError();
        return ok;
    }();
    if (!lds_ok) return hipErrorInvalidValue;
    hipLaunchKernelGGL(topk_init_kernel, dim3(1), dim3(256), 0, s, ctl, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = (int)std::min<int64_t>(std::max<int64_t>((n + 2047) / 2048, 1), 1024);
    for (int phase = 0; phase < 12; phase++) {
        hipLaunchKernelGGL(topk_hist_kernel, dim3(grid), dim3(256), 0, s, cost, n, ctl, phase);
        hipLaunchKernelGGL(topk_pick_kernel, dim3(1), dim3(256), 0, s, ctl, phase);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(topk_gather_kernel, dim3(grid), dim3(256), 0, s, cost, n, ctl, sel_cost, sel_pos);
    int P = 1;
    while (P < k) P <<= 1;
    hipLaunchKernelGGL(topk_sort_kernel, dim3(1), dim3(1024), (size_t)12 * P, s, sel_cost, sel_pos, (int32_t)k, table,
                       width, out_rows, out_cost);
    return hipGetLastError();
}

int sort_max_lds_bytes() {
    static int cached = -1;
    if (cached < 0) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 65536;
        v -= (int)sizeof(SortJob) + 64;  // static shared of the kernel
        if (v > 160 * 1024 - 512) v = 160 * 1024 - 512;
        if (v > 64 * 1024 - 512) {
            bool ok = true;
            for (const void* f : {(const void*)sort_lds_kernel, (const void*)sort_chunk_kernel})
                ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                v = 64 * 1024 - 512;
            }
        }
        cached = v;
    }
    return cached;
}

hipError_t launch_sort_lds(const SortLaunch& a, int grid, int threads, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(sort_lds_kernel, dim3(grid), dim3(threads), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_sort_merge_tier(const SortLaunch& a, int passes, hipStream_t s) {
    // one 160 KB tile per CU: 1024 threads share each network
    hipLaunchKernelGGL(sort_chunk_kernel, dim3(256), dim3(1024), a.lds_bytes, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SortLaunch m = a;
    for (int p = 0; p < passes; p++) {
        m.pass = p;
        hipLaunchKernelGGL(sort_merge_kernel, dim3(1024), dim3(kSortBlock), 0, s, m);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sort_gather_kernel, dim3(1024), dim3(kSortBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fills, offsets, column gathers
// ---------------------------------------------------------------------------

__global__ void slice_rows_kernel(const int32_t* offs, int32_t v0, int32_t v1, int64_t* n, int64_t* row0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *row0 = offs[v0];
        *n = (int64_t)offs[v1] - offs[v0];
    }
}

hipError_t launch_slice_rows(const int32_t* offs, int32_t v0, int32_t v1, int64_t* n, int64_t* row0, hipStream_t s) {
    hipLaunchKernelGGL(slice_rows_kernel, dim3(1), dim3(64), 0, s, offs, v0, v1, n, row0);
    return hipGetLastError();
}

__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// zeros, except p[at] = v
__global__ void clear_set_u64_kernel(uint64_t* p, int64_t n, int64_t at, uint64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = i == at ? v : 0ull;
}
__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void iota_i32_kernel(int32_t* p, int32_t start, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = start + (int32_t)i;
}

static int grid_for(int64_t n, int block, int max_grid = 4096) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > max_grid) g = max_grid;
    return (int)g;
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_clear_set_u64(uint64_t* p, int64_t n, int64_t at, uint64_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(clear_set_u64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, at, v);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_iota_i32(int32_t* p, int32_t start, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, start, n);
    return hipGetLastError();
}

// offs[v] = first row whose key >= v (keys ascending), v in [0, n_vertices].
__global__ void offsets_kernel(const int32_t* key, const int64_t* n_rows, int64_t cap, int32_t nv, int32_t* offs) {
    int64_t n = *n_rows;
    n = n > cap ? cap : n;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= nv; v += (int64_t)gridDim.x * blockDim.x)
        offs[v] = (int32_t)lower_bound_i32(key, n, (int32_t)v);
}

hipError_t launch_offsets(const int32_t* key, const int64_t* n_rows, int64_t cap, int32_t n_vertices, int32_t* offs,
                          hipStream_t s) {
    hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)n_vertices + 1, 256)), dim3(256), 0, s, key, n_rows,
                       cap, n_vertices, offs);
    return hipGetLastError();
}

struct ColMap {
    int32_t c[kMaxMotif];
};

__global__ void gather_cols_kernel(const int32_t* in, int64_t in_stride, const int64_t* n_rows, int64_t cap,
                                   ColMap map, int32_t ncols, int32_t* out, int64_t out_stride) {
    int64_t n = *n_rows;
    n = n > cap ? cap : n;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        for (int j = 0; j < ncols; j++) out[(int64_t)j * out_stride + r] = in[(int64_t)map.c[j] * in_stride + r];
}

hipError_t launch_gather_cols(const int32_t* in, int64_t in_stride, const int64_t* n_rows, int64_t cap,
                              const int32_t* colmap, int32_t ncols, int32_t* out, int64_t out_stride,
                              hipStream_t s) {
    ColMap m;
    for (int j = 0; j < kMaxMotif; j++) m.c[j] = j < ncols ? colmap[j] : 0;
    hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_for(cap, 256)), dim3(256), 0, s, in, in_stride, n_rows, cap, m,
                       ncols, out, out_stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// data-graph ingest: drop loops, add both orientations, sort + dedup lists
// ---------------------------------------------------------------------------

__global__ void ingest_count_kernel(const int32_t* edges, int64_t m, int32_t n, int32_t* deg, int32_t* err) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) {
            atomicOr(err, 1);
            continue;
        }
        if (u == v) continue;
        atomicAdd(&deg[u], 1);
        atomicAdd(&deg[v], 1);
    }
}

hipError_t launch_ingest_count(const int32_t* edges, int64_t m, int32_t n, int32_t* deg, int32_t* err,
                               hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(ingest_count_kernel, dim3(grid_for(m, 256)), dim3(256), 0, s, edges, m, n, deg, err);
    return hipGetLastError();
}

// Exclusive scan of int32 values (sums must fit int32; checked by the host).
// out_excl has n+1 entries; out_excl[n] = total.  Single pass: tiles of
// 256 * ITEMS values (each thread a run of ITEMS, 16-byte loads and stores
// where whole and aligned), decoupled look-back between tiles.  Long inputs
// take 16 per thread: the tile's look-back round, not its bytes, sets the
// pace at 4.
constexpr int kScanBlock = 256;
template <int ITEMS>
__global__ __launch_bounds__(kScanBlock) void scan_i32_kernel(const int32_t* in, int32_t* out, int64_t n,
                                                              int64_t* total, uint64_t* status, uint64_t* ticket,
                                                              uint32_t epoch, const WaitCtl wc) {
    constexpr int NW = kScanBlock / 64;
    constexpr int TILE = kScanBlock * ITEMS;
    __shared__ int64_t s_tile, s_base;
    __shared__ int32_t s_wsum[NW], s_wexcl[NW];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t n_tiles = (n + TILE - 1) / TILE;
    for (;;) {
        if (tid == 0) s_tile = (int64_t)atomicAdd((unsigned long long*)ticket, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= n_tiles) {
            if (tile == 0 && tid == 0) {
                out[0] = 0;
                *total = 0;
            }
            break;
        }
        int32_t vals[ITEMS];
        int32_t sum = 0;
        const int64_t base_i = tile * TILE + (int64_t)tid * ITEMS;
        const bool whole = base_i + ITEMS <= n;
        if (whole && ((uintptr_t)(in + base_i) & 15) == 0) {
#pragma unroll
            for (int q = 0; q < ITEMS / 4; q++) {
                const int4 v = *(const int4*)(in + base_i + 4 * q);
                vals[4 * q] = v.x;
                vals[4 * q + 1] = v.y;
                vals[4 * q + 2] = v.z;
                vals[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; i++) vals[i] = (base_i + i < n) ? in[base_i + i] : 0;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; i++) sum += vals[i];
        int32_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_wsum[wid] = x;
        __syncthreads();
        if (wid == 0) {
            const int32_t w = lane < NW ? s_wsum[lane] : 0;
            int32_t wi = w;
#pragma unroll
            for (int o = 1; o < NW; o <<= 1) {
                const int32_t y = __shfl_up(wi, o, 64);
                if (lane >= o) wi += y;
            }
            if (lane < NW) s_wexcl[lane] = wi - w;
            const int32_t tot = __shfl(wi, NW - 1, 64);
            // a look-back that gave up counts the missing prefix as 0: the
            // offsets come out smaller than the true ones, so what later
            // kernels index with them stays in bounds until the host sees the
            // abort word and fails the build
            int64_t excl = lookback_wave(status, epoch, tile, (uint64_t)tot, lane, wc, -1, -1);
            if (excl < 0) excl = 0;
            if (lane == 0) {
                s_base = excl;
                if (tile == n_tiles - 1) {
                    out[n] = (int32_t)(excl + tot);
                    *total = excl + tot;
                }
            }
        }
        __syncthreads();
        int64_t run = s_base + s_wexcl[wid] + (x - sum);
        if (whole && ((uintptr_t)(out + base_i) & 15) == 0) {
#pragma unroll
            for (int q = 0; q < ITEMS / 4; q++) {
                int4 v;
                v.x = (int32_t)run;
                run += vals[4 * q];
                v.y = (int32_t)run;
                run += vals[4 * q + 1];
                v.z = (int32_t)run;
                run += vals[4 * q + 2];
                v.w = (int32_t)run;
                run += vals[4 * q + 3];
                *(int4*)(out + base_i + 4 * q) = v;
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (base_i + i < n) out[base_i + i] = (int32_t)run;
                run += vals[i];
            }
        }
    }
}

hipError_t launch_scan_i32(const int32_t* in, int32_t* out_excl, int64_t n, int64_t* total, uint64_t* status,
                           uint64_t* tickets, uint32_t epoch, const WaitCtl& w, hipStream_t s) {
    if (n >= ((int64_t)1 << 20)) {
        const int64_t tiles = (n + kScanBlock * 16 - 1) / (kScanBlock * 16);
        hipLaunchKernelGGL(scan_i32_kernel<16>, dim3(grid_for(tiles, 1, 1024)), dim3(kScanBlock), 0, s, in, out_excl,
                           n, total, status, tickets + epoch, epoch, w);
    } else {
        const int64_t tiles = (n + kScanBlock * 4 - 1) / (kScanBlock * 4);
        hipLaunchKernelGGL(scan_i32_kernel<4>, dim3(grid_for(tiles, 1, 1024)), dim3(kScanBlock), 0, s, in, out_excl,
                           n, total, status, tickets + epoch, epoch, w);
    }
    return hipGetLastError();
}

// Several device ranges copied into pinned host memory by one kernel (the
// stores reach host memory over the fabric; the system-scope fence makes
// them visible before the kernel completes), in place of one copy each.
__global__ void gather_to_host_kernel(const HostGather g) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int q = 0; q < g.n; q++) {
        const uint32_t* src = (const uint32_t*)g.src[q];
        uint32_t* dst = (uint32_t*)g.dst[q];
        const int64_t words = g.bytes[q] / 4;
        for (int64_t i = t0; i < words; i += stride) dst[i] = src[i];
    }
    __threadfence_system();
}

hipError_t launch_gather_to_host(const HostGather& g, hipStream_t s) {
    int64_t words = 0;
    for (int q = 0; q < g.n; q++) words = std::max<int64_t>(words, g.bytes[q] / 4);
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_to_host_kernel, dim3(grid_for(words, 256, 64)), dim3(256), 0, s, g);
    return hipGetLastError();
}

__global__ void ingest_scatter_kernel(const int32_t* edges, int64_t m, int32_t n, const int32_t* ptr, int32_t* cursor,
                                      int32_t* tmp) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v || u < 0 || v < 0 || u >= n || v >= n) continue;  // range errors are flagged by the count
        tmp[ptr[u] + atomicAdd(&cursor[u], 1)] = v;
        tmp[ptr[v] + atomicAdd(&cursor[v], 1)] = u;
    }
}

hipError_t launch_ingest_scatter(const int32_t* edges, int64_t m, int32_t n, const int32_t* ptr, int32_t* cursor,
                                 int32_t* tmp, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(ingest_scatter_kernel, dim3(grid_for(m, 256)), dim3(256), 0, s, edges, m, n, ptr, cursor, tmp);
    return hipGetLastError();
}

constexpr int kSmallDeg = 64;
constexpr int kBigDegMax = 16384;

__global__ void ingest_sort_small_kernel(const int32_t* ptr, int32_t* tmp, int32_t n, int32_t* udeg, int32_t* big,
                                         int32_t* big_n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t* seg = tmp + ptr[v];
        const int32_t d = ptr[v + 1] - ptr[v];
        if (d > kSmallDeg) {
            big[atomicAdd(big_n, 1)] = (int32_t)v;
            continue;
        }
        for (int32_t i = 1; i < d; i++) {  // insertion sort
            const int32_t x = seg[i];
            int32_t j = i - 1;
            while (j >= 0 && seg[j] > x) {
                seg[j + 1] = seg[j];
                j--;
            }
            seg[j + 1] = x;
        }
        int32_t u = 0;
        for (int32_t i = 0; i < d; i++)
            if (i == 0 || seg[i] != seg[i - 1]) seg[u++] = seg[i];
        udeg[v] = u;
    }
}

hipError_t launch_ingest_sort_small(const int32_t* ptr, int32_t* tmp, int32_t n, int32_t* udeg, int32_t* big,
                                    int32_t* big_n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ingest_sort_small_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, ptr, tmp, n, udeg, big,
                       big_n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void ingest_sort_big_kernel(const int32_t* ptr, int32_t* tmp, int32_t* udeg,
                                                              const int32_t* big, const int32_t* big_n, int32_t* err) {
    __shared__ int32_t buf[kBigDegMax];
    const int tid = threadIdx.x;
    const int32_t nb = *big_n;
    for (int32_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int32_t v = big[b];
        int32_t* seg = tmp + ptr[v];
        const int32_t d = ptr[v + 1] - ptr[v];
        if (d > kBigDegMax) {
            if (tid == 0) {
                atomicOr(err, 2);
                udeg[v] = 0;
            }
            continue;
        }
        int P = 1;
        while (P < d) P <<= 1;
        for (int i = tid; i < P; i += 256) buf[i] = i < d ? seg[i] : INT_MAX;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = tid; t < (P >> 1); t += 256) {
                    const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
                    const bool asc = (lo & size) == 0;
                    const int32_t x = buf[lo], y = buf[hi];
                    if ((x > y) == asc) {
                        buf[lo] = y;
                        buf[hi] = x;
                    }
                }
                __syncthreads();
            }
        if (tid == 0) {  // serial dedup write-back (rare path)
            int32_t u = 0;
            for (int32_t i = 0; i < d; i++)
                if (i == 0 || buf[i] != buf[i - 1]) seg[u++] = buf[i];
            udeg[v] = u;
        }
        __syncthreads();
    }
}

hipError_t launch_ingest_sort_big(const int32_t* ptr, int32_t* tmp, int32_t* udeg, const int32_t* big,
                                  const int32_t* big_n, int32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(ingest_sort_big_kernel, dim3(64), dim3(256), 0, s, ptr, tmp, udeg, big, big_n, err);
    return hipGetLastError();
}

__global__ void ingest_compact_kernel(const int32_t* tmp_ptr, const int32_t* tmp, const int32_t* row_ptr, int32_t n,
                                      int32_t* col, int32_t* src, int32_t* max_deg) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = row_ptr[v], d = row_ptr[v + 1] - row_ptr[v];
        const int32_t* s = tmp + tmp_ptr[v];
        for (int32_t i = 0; i < d; i++) {
            col[b + i] = s[i];
            src[b + i] = (int32_t)v;
        }
        atomicMax(max_deg, d);
    }
}

hipError_t launch_ingest_compact(const int32_t* tmp_ptr, const int32_t* tmp, const int32_t* row_ptr, int32_t n,
                                 int32_t* col, int32_t* src, int32_t* max_deg, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ingest_compact_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, tmp_ptr, tmp, row_ptr, n, col,
                       src, max_deg);
    return hipGetLastError();
}

// ---- key groups ordered by a second position: one thread per group,
// stable insertion sort (groups of at most kGroupSortMax rows)
__global__ void group_sort_kernel(const int32_t* offs, int32_t n, int64_t stride, int32_t size, int32_t sec,
                                  int32_t* data) {
    const int32_t* key = data + (int64_t)sec * stride;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = offs[v], b = offs[v + 1];
        if (b - a < 2 || b - a > kGroupSortMax) continue;
        for (int32_t i = a + 1; i < b; i++) {
            int32_t row[6];
#pragma unroll
            for (int q = 0; q < 6; q++) row[q] = q < size ? data[(int64_t)q * stride + i] : 0;
            const int32_t x = key[i];
            int32_t j = i - 1;
            while (j >= a && key[j] > x) {
#pragma unroll
                for (int q = 0; q < 6; q++)
                    if (q < size) data[(int64_t)q * stride + j + 1] = data[(int64_t)q * stride + j];
                j--;
            }
#pragma unroll
            for (int q = 0; q < 6; q++)
                if (q < size) data[(int64_t)q * stride + j + 1] = row[q];
        }
    }
}

hipError_t launch_group_sort(const int32_t* offs, int32_t n, int64_t stride, int32_t size, int32_t sec, int32_t* data,
                             hipStream_t s) {
    if (n <= 0 || size > 6 || sec < 0 || sec >= size) return hipSuccess;
    hipLaunchKernelGGL(group_sort_kernel, dim3(grid_for(n, 64)), dim3(64), 0, s, offs, n, stride, size, sec, data);
    return hipGetLastError();
}

// Order every key group (rows [offs[v], offs[v+1]) of the SoA table `in`,
// `size` columns of stride `stride`) by column `sec`, stably, into `out`
// (same offsets): one workgroup per key vertex sorts (value, position) pairs
// with a bitonic network in LDS and writes every column permuted.  Groups of
// more than cap rows (the dynamic LDS holds cap pairs, a power of two) are
// copied unchanged.
__global__ __launch_bounds__(256) void group_sort_lds_kernel(const int32_t* offs, int32_t n, int64_t stride,
                                                             int32_t size, int32_t sec, const int32_t* in,
                                                             int32_t* out, int32_t cap) {
    extern __shared__ uint64_t key[];
    const int tid = threadIdx.x, nt = (int)blockDim.x;
    for (int32_t v = blockIdx.x; v < n; v += gridDim.x) {
        const int32_t a = offs[v], len = offs[v + 1] - offs[v];
        if (len <= 0) continue;
        if (len == 1 || len > cap) {
            for (int64_t e = tid; e < (int64_t)len * size; e += nt) {
                const int64_t i = e / size;
                const int q = (int)(e - i * size);
                out[(int64_t)a * size + e] = in[(int64_t)q * stride + a + i];
            }
            continue;
        }
        int P = 1;
        while (P < len) P <<= 1;
        const int32_t* kc = in + (int64_t)sec * stride + a;
        for (int i = tid; i < P; i += nt) key[i] = i < len ? (((uint64_t)(uint32_t)kc[i] << 32) | (uint32_t)i) : ~0ull;
        __syncthreads();
        for (int sz = 2; sz <= P; sz <<= 1) {
            for (int st = sz >> 1; st > 0; st >>= 1) {
                for (int t = tid; t < (P >> 1); t += nt) {
                    const int lo = 2 * t - (t & (st - 1)), hi = lo + st;
                    const uint64_t x = key[lo], y = key[hi];
                    if ((x > y) == ((lo & sz) == 0)) {
                        key[lo] = y;
                        key[hi] = x;
                    }
                }
                __syncthreads();
            }
        }
        // row-major: consecutive threads write consecutive words of the rows
        for (int32_t e = tid; e < len * size; e += nt) {
            const int32_t i = e / size, q = e - i * size;
            out[(int64_t)a * size + e] = in[(int64_t)q * stride + a + (uint32_t)key[i]];
        }
        __syncthreads();  // key[] is refilled for the next group
    }
}

// run starts of a row-major table ordered by (column 0, column sec)
__global__ void run_flags_kernel(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, int32_t* flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t* r = aos + i * size;
        flags[i] = (i == 0 || r[0] != r[-size] || r[sec] != r[sec - size]) ? 1 : 0;
    }
}

__global__ void run_fill_kernel(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, const int32_t* flags,
                                const int32_t* idx, int32_t* run_far, int32_t* run_start) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
        if (flags[i]) {
            run_far[idx[i]] = aos[i * size + sec];
            run_start[idx[i]] = (int32_t)i;
        }
}

__global__ void run_offs_kernel(const int32_t* offs, int32_t n, int64_t rows, const int32_t* idx,
                                const int64_t* total, int32_t* run_offs) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = offs[v];
        run_offs[v] = r < rows ? idx[r] : (int32_t)*total;
    }
}

hipError_t launch_run_flags(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, int32_t* flags,
                            hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(run_flags_kernel, dim3(grid_for(rows, 256)), dim3(256), 0, s, aos, rows, size, sec, flags);
    return hipGetLastError();
}

hipError_t launch_run_fill(const int32_t* aos, int64_t rows, int32_t size, int32_t sec, const int32_t* flags,
                           const int32_t* idx, int32_t* run_far, int32_t* run_start, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(run_fill_kernel, dim3(grid_for(rows, 256)), dim3(256), 0, s, aos, rows, size, sec, flags, idx,
                       run_far, run_start);
    return hipGetLastError();
}

hipError_t launch_run_offs(const int32_t* offs, int32_t n, int64_t rows, const int32_t* idx, const int64_t* total,
                           int32_t* run_offs, hipStream_t s) {
    hipLaunchKernelGGL(run_offs_kernel, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, s, offs, n, rows, idx,
                       total, run_offs);
    return hipGetLastError();
}

hipError_t launch_group_sort_lds(const int32_t* offs, int32_t n, int64_t stride, int32_t size, int32_t sec,
                                 const int32_t* in, int32_t* out, int32_t cap, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (sec < 0 || sec >= size || cap <= 0 || cap > kGroupSortLds || (cap & (cap - 1))) return hipErrorInvalidValue;
    // LDS sized by the largest group, not by the kernel's limit: more
    // workgroups resident per CU when the groups are small
    hipLaunchKernelGGL(group_sort_lds_kernel, dim3(n < 16384 ? n : 16384), dim3(256), sizeof(uint64_t) * (size_t)cap,
                       s, offs, n, stride, size, sec, in, out, cap);
    return hipGetLastError();
}

// ---- the claw table (M4-1: centre 0, leaves 1..3) straight from the CSR.
// Keyed at the centre (key_pos 0) the rows of vertex v are (v, a, b, d) for
// every ordered triple of distinct neighbours of v; keyed at a leaf
// (key_pos 1) they are (c, v, a, b) for every neighbour c of v and ordered
// pair (a, b) of distinct neighbours of c other than v.  Either way every
// embedding of the claw appears once, grouped by the key position's image.
__global__ void claw_count_kernel(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos, int32_t* cnt) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        if (key_pos == 0) {
            const int64_t d = rp[v + 1] - rp[v];
            c = d * (d - 1) * (d - 2);
        } else {
            for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
                const int32_t u = col[i];
                const int64_t d = rp[u + 1] - rp[u];
                c += (d - 1) * (d - 2);
            }
        }
        cnt[v] = (int32_t)c;  // the host checked that the total fits
    }
}

__global__ void claw_fill_kernel(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos,
                                 const int32_t* offs, int64_t stride, int32_t* data) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = offs[v];
        auto put = [&](int32_t x0, int32_t x1, int32_t x2, int32_t x3) {
            data[r] = x0;
            data[stride + r] = x1;
            data[2 * stride + r] = x2;
            data[3 * stride + r] = x3;
            r++;
        };
        if (key_pos == 0) {
            for (int32_t i = rp[v]; i < rp[v + 1]; i++)
                for (int32_t j = rp[v]; j < rp[v + 1]; j++) {
                    if (j == i) continue;
                    for (int32_t l = rp[v]; l < rp[v + 1]; l++)
                        if (l != i && l != j) put((int32_t)v, col[i], col[j], col[l]);
                }
        } else {
            for (int32_t i = rp[v]; i < rp[v + 1]; i++) {
                const int32_t c = col[i];
                for (int32_t j = rp[c]; j < rp[c + 1]; j++) {
                    if (col[j] == v) continue;
                    for (int32_t l = rp[c]; l < rp[c + 1]; l++)
                        if (l != j && col[l] != v) put(c, (int32_t)v, col[j], col[l]);
                }
            }
        }
    }
}

hipError_t launch_claw_count(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos, int32_t* cnt,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(claw_count_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, rp, col, n, key_pos, cnt);
    return hipGetLastError();
}

hipError_t launch_claw_fill(const int32_t* rp, const int32_t* col, int32_t n, int32_t key_pos, const int32_t* offs,
                            int64_t stride, int32_t* data, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(claw_fill_kernel, dim3(grid_for(n, 64)), dim3(64), 0, s, rp, col, n, key_pos, offs, stride,
                       data);
    return hipGetLastError();
}

__global__ void bitmap_set_kernel(const int32_t* src, const int32_t* col, const int64_t* nnz_dev, int32_t wpr,
                                  uint32_t* bm) {
    const int64_t nnz = *nnz_dev;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e], w = col[e];
        atomicOr(&bm[(size_t)u * (size_t)wpr + (size_t)(w >> 5)], 1u << (w & 31));
    }
}

// A 4-cycle v-u-w-u'-v exists iff some vertex v has two distinct neighbours
// with a common neighbour other than v.  Thread per vertex: every pair of its
// neighbours, their ascending lists merged.  flags[0] |= 1 when one is found;
// flags[1] |= 1 when a vertex has more than kC4MaxDegree neighbours (then the
// answer is left to the caller).
constexpr int kC4MaxDegree = 16;
// Degree <= 4 around v (lattices): the neighbours' lists in registers,
// four dependent load rounds, every pair compared.  Returns -1 when some
// neighbour has more than 4 neighbours (the merge walk decides then).
__device__ __forceinline__ int c4_small(const int32_t* row_ptr, const int32_t* col, int32_t v, int32_t b, int32_t d) {
    int32_t u[4];
#pragma unroll
    for (int i = 0; i < 4; i++) u[i] = i < d ? col[b + i] : -1;
    int32_t rs[4], du[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        rs[i] = u[i] >= 0 ? row_ptr[u[i]] : 0;
        du[i] = u[i] >= 0 ? row_ptr[u[i] + 1] - rs[i] : 0;
    }
    bool wide = false;
#pragma unroll
    for (int i = 0; i < 4; i++) wide |= du[i] > 4;
    if (wide) return -1;
    int32_t w[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int32_t x = j < du[i] ? col[rs[i] + j] : -1;
            w[i][j] = x == v ? -1 : x;  // v itself closes nothing
        }
    bool found = false;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int i2 = i + 1; i2 < 4; i2++)
#pragma unroll
            for (int j = 0; j < 4; j++)
#pragma unroll
                for (int j2 = 0; j2 < 4; j2++) found |= w[i][j] >= 0 && w[i][j] == w[i2][j2];
    return found ? 1 : 0;
}

__global__ void c4_check_kernel(const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t* flags) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = row_ptr[v], e = row_ptr[v + 1];
        if (e - b > kC4MaxDegree) {
            atomicOr(&flags[1], 1);
            continue;
        }
        if (e - b <= 4) {
            const int r = c4_small(row_ptr, col, (int32_t)v, b, e - b);
            if (r == 1) atomicOr(&flags[0], 1);
            if (r >= 0) continue;
        }
        bool found = false;
        for (int32_t i = b; i < e && !found; i++) {
            const int32_t u1 = col[i];
            for (int32_t j = i + 1; j < e && !found; j++) {
                const int32_t u2 = col[j];
                int32_t p = row_ptr[u1], pe = row_ptr[u1 + 1], q = row_ptr[u2], qe = row_ptr[u2 + 1];
                while (p < pe && q < qe) {
                    const int32_t a = col[p], c = col[q];
                    if (a == c) {
                        if (a != (int32_t)v) {
                            found = true;
                            break;
                        }
                        p++;
                        q++;
                    } else if (a < c) {
                        p++;
                    } else {
                        q++;
                    }
                }
            }
        }
        if (found) atomicOr(&flags[0], 1);
    }
}

hipError_t launch_c4_check(const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(c4_check_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, row_ptr, col, n, flags);
    return hipGetLastError();
}

hipError_t launch_bitmap_set(const int32_t* src, const int32_t* col, const int64_t* nnz_dev, int64_t nnz_max,
                             int32_t wpr, uint32_t* bitmap, hipStream_t s) {
    if (nnz_max <= 0) return hipSuccess;
    hipLaunchKernelGGL(bitmap_set_kernel, dim3(grid_for(nnz_max, 256)), dim3(256), 0, s, src, col, nnz_dev, wpr,
                       bitmap);
    return hipGetLastError();
}

}  // namespace dm
