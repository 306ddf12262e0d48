// HIP kernels for gfx950 (wave64).  Everything here is integer table work:
// joins, filters, compaction, sorting and graph ingest.  None of it is a dense
// contraction, so nothing uses MFMA; the kernels are bound by HBM bandwidth
// (large tables) or by launch latency (small ones).
#include <climits>

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

// Decoupled look-back (single-pass chained scan) executed by one full wave.
// Tiles are claimed in ticket order by running workgroups, so every
// predecessor of `tile` is owned by a workgroup that is already running and
// will publish; the wait always ends.  Returns the exclusive prefix.
__device__ int64_t lookback_wave(uint64_t* status, uint32_t epoch, int64_t tile, uint64_t agg, int lane) {
    if (tile == 0) {
        if (lane == 0) st_relaxed(&status[0], lb_pack(epoch, 2, agg));
        return 0;
    }
    if (lane == 0) st_relaxed(&status[tile], lb_pack(epoch, 1, agg));
    uint64_t excl = 0;
    int64_t j = tile - 1;
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

// ---------------------------------------------------------------------------
// expand-join-filter (one iteration of the join-and-filter loop)
// ---------------------------------------------------------------------------

template <int CMAX>
__device__ __forceinline__ int32_t old_val(const EjfArgs& a, const int32_t (&v)[CMAX], int c, int64_t row) {
    if (!a.in) return v[0];
    return a.in[(int64_t)c * a.in_stride + row];
}

__device__ __forceinline__ int32_t pick_new(const int32_t (&nv)[kMaxMotif], int t) {
    int32_t r = -1;
#pragma unroll
    for (int i = 0; i < kMaxMotif; i++) r = (i == t) ? nv[i] : r;
    return r;
}

// Does motif row m extend input row `row` (values v) into a valid partial
// embedding?  Join keys (the index lookup plus eq checks), injectivity of the
// new values against the row, and the step's explicit edge checks.
template <int CMAX>
__device__ __forceinline__ bool ejf_accept(const EjfArgs& a, const int32_t (&v)[CMAX], int64_t row, int32_t m,
                                           int32_t (&nv)[kMaxMotif]) {
    const StepDesc& st = a.st;
    if (st.motif >= 0) {
        for (int e = 0; e < st.n_eq; e++) {
            if (a.tbl.col[st.eq_pos[e]][m] != old_val(a, v, st.eq_col[e], row)) return false;
        }
#pragma unroll
        for (int t = 0; t < kMaxMotif; t++) {
            if (t < st.n_new) {
                const int32_t x = a.tbl.col[st.new_pos[t]][m];
                nv[t] = x;
                bool clash = false;
#pragma unroll
                for (int c = 0; c < CMAX; c++) clash |= (v[c] == x);
                if (clash) return false;
            }
        }
    }
    for (int e = 0; e < st.n_edge; e++) {
        const int ca = st.edge_a[e], cb = st.edge_b[e];
        const int32_t va = ca < st.c_in ? old_val(a, v, ca, row) : pick_new(nv, ca - st.c_in);
        const int32_t vb = cb < st.c_in ? old_val(a, v, cb, row) : pick_new(nv, cb - st.c_in);
        if (!adjacent(a.g, va, vb)) return false;
    }
    return true;
}

template <int BLOCK>
struct TileShared {
    static constexpr int CH = 8 * BLOCK;  // output rows staged per write pass
    int64_t base;
    int32_t total;
    int32_t wsum[BLOCK / 64];
    int32_t wexcl[BLOCK / 64];
    int32_t mrow[CH];   // motif row of each staged output row
    uint8_t src[CH];    // input row (lane of the tile) of each staged output row
};

// One tile (BLOCK consecutive input rows) of a join-filter step: count the
// surviving candidates of every row, take this tile's output offset from the
// look-back chain, then write the surviving rows in input order.  In hash
// mode the survivors only feed the per-thread (count, sum, xor) accumulators.
template <int CMAX, int BLOCK>
__device__ __forceinline__ void ejf_tile(const EjfArgs& a, int64_t tile, int64_t n_in, int64_t n_tiles,
                                         TileShared<BLOCK>& sh, uint64_t& h_cnt, uint64_t& h_sum,
                                         uint64_t& h_xor) {
    constexpr int NW = BLOCK / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const StepDesc& st = a.st;
    const int64_t row = tile * BLOCK + tid;
    const bool valid = row < n_in;
    int32_t v[CMAX];
#pragma unroll
    for (int c = 0; c < CMAX; c++) v[c] = -1;
    if (valid) {
        if (a.in) {
#pragma unroll
            for (int c = 0; c < CMAX; c++)
                if (c < st.c_in) v[c] = a.in[(int64_t)c * a.in_stride + row];
        } else {
            v[0] = a.id_begin + (int32_t)row;
        }
    }
    int32_t lo = 0, hi = 0;
    if (valid) {
        if (st.motif >= 0) {
            const int32_t key = a.in ? a.in[(int64_t)st.key_col * a.in_stride + row] : v[0];
            lo = a.tbl.offs[key];
            hi = a.tbl.offs[key + 1];
        } else {
            hi = 1;  // filter-only step: the row itself is the one candidate
        }
    }
    int32_t nv[kMaxMotif];
#pragma unroll
    for (int t = 0; t < kMaxMotif; t++) nv[t] = -1;

    if (a.mode == EJF_HASH) {
        uint64_t inner_old = 0;
        if (valid) {
#pragma unroll
            for (int c = 0; c < CMAX; c++)
                if (c < st.c_in) inner_old += mix64(((uint64_t)a.pv[c] << 32) | (uint32_t)v[c]);
        }
        for (int32_t m = lo; m < hi; m++) {
            if (!ejf_accept<CMAX>(a, v, row, m, nv)) continue;
            uint64_t inner = inner_old;
#pragma unroll
            for (int t = 0; t < kMaxMotif; t++)
                if (t < st.n_new) inner += mix64(((uint64_t)a.pv[st.c_in + t] << 32) | (uint32_t)nv[t]);
            const uint64_t h = mix64(inner);
            h_cnt++;
            h_sum += h;
            h_xor ^= h;
        }
        return;
    }

    uint64_t mask = 0;
    int32_t cnt = 0;
    for (int32_t m = lo; m < hi; m++) {
        if (ejf_accept<CMAX>(a, v, row, m, nv)) {
            if (m - lo < 64) mask |= 1ull << (m - lo);
            cnt++;
        }
    }
    // block-wide exclusive scan of per-row survivor counts
    int32_t x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh.wsum[wid] = x;
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
        const int64_t excl = lookback_wave(a.status, a.epoch, tile, (uint64_t)total, lane);
        if (lane == 0) {
            sh.base = excl;
            sh.total = total;
            if (tile == n_tiles - 1) *a.n_out = excl + total;
            if (excl + total > a.out_cap) *a.overflow = 1;
        }
    }
    __syncthreads();
    // Write phase.  Survivors are staged in LDS in output order as (input
    // lane, motif row); then each thread assembles whole output rows and
    // writes them column by column, so every store of a wave covers
    // consecutive elements of one column (coalesced), instead of each lane
    // scattering its own survivors.
    constexpr int CH = TileShared<BLOCK>::CH;
    const int32_t local0 = sh.wexcl[wid] + (x - cnt);
    const int32_t total = sh.total;
    const int64_t base = sh.base;
    const int c_in = st.c_in, n_new = st.motif >= 0 ? st.n_new : 0;
    const int64_t row0 = tile * BLOCK;
    // each thread's candidate cursor survives across passes, so every
    // candidate is visited once however many passes the tile needs
    int32_t m_cur = lo, r_cur = 0;
    for (int32_t w0 = 0; w0 < total; w0 += CH) {
        while (r_cur < cnt && m_cur < hi) {
            const int32_t li = local0 + r_cur;
            if (li >= w0 + CH) break;  // belongs to a later pass
            const int32_t m = m_cur++;
            const bool ok =
                (m - lo < 64) ? (bool)((mask >> (m - lo)) & 1ull) : ejf_accept<CMAX>(a, v, row, m, nv);
            if (!ok) continue;
            sh.src[li - w0] = (uint8_t)tid;
            sh.mrow[li - w0] = m;
            r_cur++;
        }
        __syncthreads();
        const int32_t nrows = (total - w0 < CH) ? (total - w0) : CH;
        const int64_t obase = base + w0;
        for (int32_t o = tid; o < nrows; o += BLOCK) {
            const int64_t orow = obase + o;
            if (orow >= a.out_cap) break;
            const int64_t irow = row0 + sh.src[o];
            const int32_t m = sh.mrow[o];
            if (a.in) {
                for (int c = 0; c < c_in; c++)
                    a.out[(int64_t)c * a.out_stride + orow] = a.in[(int64_t)c * a.in_stride + irow];
            } else {
                a.out[orow] = a.id_begin + (int32_t)irow;
            }
            for (int t = 0; t < n_new; t++)
                a.out[(int64_t)(c_in + t) * a.out_stride + orow] = a.tbl.col[st.new_pos[t]][m];
        }
        __syncthreads();
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
// until the input is exhausted.
template <int CMAX, int BLOCK>
__global__ __launch_bounds__(BLOCK) void ejf_kernel(const EjfArgs a) {
    __shared__ TileShared<BLOCK> sh;
    __shared__ int64_t s_tile;
    __shared__ uint64_t s_red[3][BLOCK / 64];
    const int tid = threadIdx.x;
    const int64_t n_in = a.in ? clamp_rows(*a.n_in, a.in_cap) : (int64_t)a.id_count;
    const int64_t n_tiles = (n_in + BLOCK - 1) / BLOCK;
    uint64_t h_cnt = 0, h_sum = 0, h_xor = 0;
    for (;;) {
        if (tid == 0) s_tile = (int64_t)atomicAdd((unsigned long long*)a.ticket, 1ull);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= n_tiles) {
            if (a.mode == EJF_WRITE && tile == 0 && tid == 0) *a.n_out = 0;
            break;
        }
        ejf_tile<CMAX, BLOCK>(a, tile, n_in, n_tiles, sh, h_cnt, h_sum, h_xor);
    }
    if (a.mode == EJF_HASH) hash_flush<BLOCK>(a.hash_acc, h_cnt, h_sum, h_xor, s_red);
}

template <int CMAX>
static hipError_t launch_ejf_c(const EjfArgs& a, int block, int grid, hipStream_t s) {
    switch (block) {
        case 64: hipLaunchKernelGGL((ejf_kernel<CMAX, 64>), dim3(grid), dim3(64), 0, s, a); break;
        case 128: hipLaunchKernelGGL((ejf_kernel<CMAX, 128>), dim3(grid), dim3(128), 0, s, a); break;
        default: hipLaunchKernelGGL((ejf_kernel<CMAX, 256>), dim3(grid), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_ejf(const EjfArgs& a, int block, int grid, hipStream_t s) {
    const int c = a.st.c_in;
    if (c <= 8) return launch_ejf_c<8>(a, block, grid, s);
    if (c <= 16) return launch_ejf_c<16>(a, block, grid, s);
    if (c <= 32) return launch_ejf_c<32>(a, block, grid, s);
    if (c <= 64) return launch_ejf_c<64>(a, block, grid, s);
    return launch_ejf_c<128>(a, block, grid, s);
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

template <int CMAX>
__device__ void batch_tile_dispatch(const EjfArgs& a, int64_t tile, int64_t n_in, int64_t n_tiles,
                                    TileShared<64>& sh, uint64_t& hc, uint64_t& hs, uint64_t& hx) {
    const int c = a.st.c_in;
    if (CMAX >= 64 && c > 32) ejf_tile<(CMAX >= 64 ? 64 : CMAX), 64>(a, tile, n_in, n_tiles, sh, hc, hs, hx);
    else if (CMAX >= 32 && c > 16) ejf_tile<(CMAX >= 32 ? 32 : CMAX), 64>(a, tile, n_in, n_tiles, sh, hc, hs, hx);
    else if (CMAX >= 16 && c > 8) ejf_tile<(CMAX >= 16 ? 16 : CMAX), 64>(a, tile, n_in, n_tiles, sh, hc, hs, hx);
    else ejf_tile<8, 64>(a, tile, n_in, n_tiles, sh, hc, hs, hx);
}

template <int CMAX>
__global__ __launch_bounds__(64) void batch_kernel(const BatchDev b) {
    __shared__ TileShared<64> sh;
    __shared__ EjfArgs sa;
    __shared__ uint64_t s_red[3][1];
    const int lane = threadIdx.x;
    const int N = b.n_patterns;
    int rot = (int)((blockIdx.x * 7919u) % (unsigned)(N > 0 ? N : 1));
    uint64_t hc = 0, hs = 0, hx = 0;
    for (;;) {
        // ---- find a claimable tile (whole wave scans 64 patterns at a time)
        int32_t p = -1, s = -1;
        int64_t tile = -1;
        bool all_done = false;
        for (;;) {
            bool got = false;
            for (int base = 0; base < N && !got; base += 64) {
                const int q = (rot + base + lane) % N;
                bool avail = false;
                int32_t st = 0, nt = 0;
                if (base + lane < N) {
                    // polling uses relaxed (per-location coherent) loads: an
                    // acquire here would invalidate L1 on every poll
                    st = ld_rlx_i32(&b.ctl[q].stage);
                    if (st < b.nsteps[q]) {
                        // ntiles[s] is written once (0 -> final) before stage s is
                        // published, so a nonzero value is the final one
                        nt = ld_rlx_i32(&b.ctl[q].ntiles[st]);
                        avail = ld_rlx_i32(&b.ctl[q].claim[st]) < nt;
                    }
                }
                uint64_t m = __ballot(avail);
                while (m) {
                    const int l = __ffsll((long long)m) - 1;
                    m &= m - 1;
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
            __builtin_amdgcn_s_sleep(8);
        }
        if (all_done) break;
        rot = (p + 1) % N;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // ---- stage the step's arguments in LDS
        {
            const int32_t* src = (const int32_t*)&b.args[b.first[p] + s];
            int32_t* dst = (int32_t*)&sa;
            for (int i = lane; i < (int)(sizeof(EjfArgs) / 4); i += 64) dst[i] = src[i];
        }
        __syncthreads();
        const int64_t n_in = b.ctl[p].n_in[s];
        const int64_t n_tiles = b.ctl[p].ntiles[s];
        batch_tile_dispatch<CMAX>(sa, tile, n_in, n_tiles, sh, hc, hs, hx);
        if (sa.mode == EJF_HASH) {
            hash_flush<64>(sa.hash_acc, hc, hs, hx, s_red);
            hc = hs = hx = 0;
        }
        // ---- completion: the last tile of a step publishes the next one
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) {
            const int32_t d = atomicAdd(&b.ctl[p].done[s], 1);
            if (d == n_tiles - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                BatchCtl& c = b.ctl[p];
                const int32_t ns = b.nsteps[p];
                const int64_t n_out = (sa.mode == EJF_HASH) ? 0 : __hip_atomic_load(sa.n_out, __ATOMIC_RELAXED,
                                                                                       __HIP_MEMORY_SCOPE_AGENT);
                if (s + 1 < ns && n_out > 0) {
                    const EjfArgs& nx = b.args[b.first[p] + s + 1];
                    const int64_t nn = clamp_rows(n_out, nx.in_cap);
                    c.n_in[s + 1] = nn;
                    __hip_atomic_store(&c.ntiles[s + 1], (int32_t)((nn + 63) / 64), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    st_rel_i32(&c.stage, s + 1);
                } else {
                    // last step, or nothing left: the remaining steps produce 0 rows
                    for (int q = s + 1; q < ns; q++) *b.args[b.first[p] + q].n_out = 0;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    st_rel_i32(&c.stage, ns);
                    atomicAdd(b.finished, 1);
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_batch(const BatchDev& b, int cmax, int grid, hipStream_t s) {
    if (cmax <= 8) hipLaunchKernelGGL((batch_kernel<8>), dim3(grid), dim3(64), 0, s, b);
    else if (cmax <= 16) hipLaunchKernelGGL((batch_kernel<16>), dim3(grid), dim3(64), 0, s, b);
    else if (cmax <= 32) hipLaunchKernelGGL((batch_kernel<32>), dim3(grid), dim3(64), 0, s, b);
    else hipLaunchKernelGGL((batch_kernel<64>), dim3(grid), dim3(64), 0, s, b);
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
constexpr uint32_t kSent = 0xFFFFFFFFu;

__device__ __forceinline__ bool lds_row_less(const int32_t* rows, int kp, int k, uint32_t x, uint32_t y) {
    const int32_t* a = rows + (size_t)x * kp;
    const int32_t* b = rows + (size_t)y * kp;
    for (int j = 1; j < k; j++) {
        const int32_t p = a[j], q = b[j];
        if (p != q) return p < q;
    }
    return false;
}

// Rows of kp int32 that fit an LDS tile of lds_bytes together with the
// 16-bit index array of the bitonic network (padded to a power of two).
__device__ __forceinline__ int lds_rows_of(int lds_bytes, int kp) {
    int r = lds_bytes / (4 * kp + 4);
    if (r > 65535) r = 65535;
    while (r > 0) {
        int P = 1;
        while (P < r) P <<= 1;
        if (4 * kp * r + 2 * P <= lds_bytes) break;
        r--;
    }
    return r;
}

constexpr uint16_t kSent16 = 0xFFFFu;

// Load job j into LDS (all threads), then broadcast the segment of root v.
__device__ __forceinline__ void sort_item_setup(const SortLaunch& L, int64_t item, SortJob& job, int64_t* seg) {
    const int64_t j = item / L.n_vertices;
    const int32_t v = L.v_begin + (int32_t)(item - j * L.n_vertices);
    const int32_t* src = (const int32_t*)&L.jobs[j];
    int32_t* dst = (int32_t*)&job;
    for (int i = threadIdx.x; i < (int)(sizeof(SortJob) / 4); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t n = clamp_rows(*job.n_in, job.in_cap);
        seg[0] = lower_bound_i32(job.in, n, v);
        seg[1] = lower_bound_i32(job.in, n, v + 1);
    }
    __syncthreads();
}

__global__ __launch_bounds__(kSortBlock) void sort_lds_kernel(const SortLaunch L) {
    extern __shared__ int32_t lds[];
    __shared__ SortJob job;
    __shared__ int64_t s_seg[2];
    const int tid = threadIdx.x;
    const int64_t n_items = L.list ? (int64_t)*L.list_n : (int64_t)L.n_jobs * L.n_vertices;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int64_t item = L.list ? (int64_t)L.list[it] : it;
        sort_item_setup(L, item, job, s_seg);
        const int64_t seg0 = s_seg[0], seg1 = s_seg[1];
        const int64_t L_ = seg1 - seg0;
        const int k = job.k, kp = job.kp;
        const int lds_rows = lds_rows_of(L.lds_bytes, kp);
        __syncthreads();
        if (L_ == 0 || seg0 >= job.out_rows) continue;
        if (L_ > lds_rows) {
            if (tid == 0) L.spill[atomicAdd(L.spill_n, 1)] = (int32_t)item;
            continue;
        }
        int32_t* rows = lds;
        uint16_t* idx = (uint16_t*)(lds + (size_t)lds_rows * kp);
        for (int j = 0; j < k; j++) {
            const int32_t* src = job.in + (int64_t)job.perm[j] * job.in_stride + seg0;
            for (int r = tid; r < L_; r += kSortBlock) rows[r * kp + j] = src[r];
        }
        int P = 1;
        while (P < L_) P <<= 1;
        for (int i = tid; i < P; i += kSortBlock) idx[i] = i < L_ ? (uint16_t)i : kSent16;
        __syncthreads();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = tid; t < (P >> 1); t += kSortBlock) {
                    const int lo = 2 * t - (t & (stride - 1));
                    const int hi = lo + stride;
                    const bool asc = (lo & size) == 0;
                    const uint16_t ia = idx[lo], ib = idx[hi];
                    bool gt;
                    if (ia == kSent16) gt = (ib != kSent16);
                    else if (ib == kSent16) gt = false;
                    else gt = lds_row_less(rows, kp, k, ib, ia);
                    if (gt == asc) {
                        idx[lo] = ib;
                        idx[hi] = ia;
                    }
                }
                __syncthreads();
            }
        }
        for (int r = tid + 1; r < L_; r += kSortBlock)
            if (!lds_row_less(rows, kp, k, idx[r - 1], idx[r])) atomicAdd(L.dup_count, 1);
        const int64_t Lw = (seg0 + L_ <= job.out_rows) ? L_ : (job.out_rows - seg0);
        const int64_t total = Lw * k;
        int32_t* dst = job.out + seg0 * k;
        for (int64_t e = tid; e < total; e += kSortBlock) {
            const int64_t r = e / k;
            const int j = (int)(e - r * k);
            dst[e] = rows[(size_t)idx[r] * kp + j];
        }
        __syncthreads();
    }
}

// Global-memory tier for segments larger than any LDS tile: bitonic sort of
// row indices in the job's scratch (2 * rows entries, disjoint per
// segment), comparing rows straight from the input columns.
__device__ __forceinline__ bool glb_row_less(const SortJob& a, int64_t seg0, uint32_t x, uint32_t y) {
    for (int j = 1; j < a.k; j++) {
        const int32_t* c = a.in + (int64_t)a.perm[j] * a.in_stride + seg0;
        const int32_t p = c[x], q = c[y];
        if (p != q) return p < q;
    }
    return false;
}

__global__ __launch_bounds__(kSortBlock) void sort_global_kernel(const SortLaunch L) {
    __shared__ SortJob job;
    __shared__ int64_t s_seg[2];
    const int tid = threadIdx.x;
    const int64_t n_items = (int64_t)*L.list_n;
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int64_t item = (int64_t)L.list[it];
        sort_item_setup(L, item, job, s_seg);
        const int64_t seg0 = s_seg[0], seg1 = s_seg[1];
        const int64_t L_ = seg1 - seg0;
        const int k = job.k;
        __syncthreads();
        if (L_ == 0 || seg0 >= job.out_rows) continue;
        uint32_t* idx = job.scratch_idx + 2 * seg0;
        int64_t P = 1;
        while (P < L_) P <<= 1;
        for (int64_t i = tid; i < P; i += kSortBlock) idx[i] = i < L_ ? (uint32_t)i : kSent;
        __threadfence_block();
        __syncthreads();
        for (int64_t size = 2; size <= P; size <<= 1) {
            for (int64_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (int64_t t = tid; t < (P >> 1); t += kSortBlock) {
                    const int64_t lo = 2 * t - (t & (stride - 1));
                    const int64_t hi = lo + stride;
                    const bool asc = (lo & size) == 0;
                    const uint32_t ia = idx[lo], ib = idx[hi];
                    bool gt;
                    if (ia == kSent) gt = (ib != kSent);
                    else if (ib == kSent) gt = false;
                    else gt = glb_row_less(job, seg0, ib, ia);
                    if (gt == asc) {
                        idx[lo] = ib;
                        idx[hi] = ia;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
        for (int64_t r = tid + 1; r < L_; r += kSortBlock)
            if (!glb_row_less(job, seg0, idx[r - 1], idx[r])) atomicAdd(L.dup_count, 1);
        const int64_t Lw = (seg0 + L_ <= job.out_rows) ? L_ : (job.out_rows - seg0);
        const int64_t total = Lw * k;
        int32_t* dst = job.out + seg0 * k;
        for (int64_t e = tid; e < total; e += kSortBlock) {
            const int64_t r = e / k;
            const int j = (int)(e - r * k);
            dst[e] = job.in[(int64_t)job.perm[j] * job.in_stride + seg0 + idx[r]];
        }
        __syncthreads();
    }
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
            if (hipFuncSetAttribute((const void*)sort_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, v) !=
                hipSuccess) {
                (void)hipGetLastError();
                v = 64 * 1024 - 512;
            }
        }
        cached = v;
    }
    return cached;
}

hipError_t launch_sort_lds(const SortLaunch& a, int grid, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(sort_lds_kernel, dim3(grid), dim3(kSortBlock), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_sort_global(const SortLaunch& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(sort_global_kernel, dim3(grid), dim3(kSortBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fills, offsets, column gathers
// ---------------------------------------------------------------------------

__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
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
// 1024 values, decoupled look-back between tiles.
constexpr int kScanBlock = 256, kScanItems = 4;
__global__ __launch_bounds__(kScanBlock) void scan_i32_kernel(const int32_t* in, int32_t* out, int64_t n,
                                                              int64_t* total, uint64_t* status, uint64_t* ticket) {
    constexpr int NW = kScanBlock / 64;
    constexpr int TILE = kScanBlock * kScanItems;
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
        int32_t vals[kScanItems];
        int32_t sum = 0;
        const int64_t base_i = tile * TILE + (int64_t)tid * kScanItems;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            vals[i] = (base_i + i < n) ? in[base_i + i] : 0;
            sum += vals[i];
        }
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
            const int64_t excl = lookback_wave(status, 0, tile, (uint64_t)tot, lane);
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
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (base_i + i < n) out[base_i + i] = (int32_t)run;
            run += vals[i];
        }
    }
}

hipError_t launch_scan_i32(const int32_t* in, int32_t* out_excl, int64_t n, int64_t* total, uint64_t* status,
                           uint64_t* ticket, hipStream_t s) {
    const int64_t tiles = (n + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
    hipLaunchKernelGGL(scan_i32_kernel, dim3(grid_for(tiles, 1, 1024)), dim3(kScanBlock), 0, s, in, out_excl, n,
                       total, status, ticket);
    return hipGetLastError();
}

__global__ void ingest_scatter_kernel(const int32_t* edges, int64_t m, const int32_t* ptr, int32_t* cursor,
                                      int32_t* tmp) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v) continue;
        tmp[ptr[u] + atomicAdd(&cursor[u], 1)] = v;
        tmp[ptr[v] + atomicAdd(&cursor[v], 1)] = u;
    }
}

hipError_t launch_ingest_scatter(const int32_t* edges, int64_t m, const int32_t* ptr, int32_t* cursor, int32_t* tmp,
                                 hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(ingest_scatter_kernel, dim3(grid_for(m, 256)), dim3(256), 0, s, edges, m, ptr, cursor, tmp);
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

__global__ void bitmap_set_kernel(const int32_t* src, const int32_t* col, int64_t nnz, int32_t wpr, uint32_t* bm) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e], w = col[e];
        atomicOr(&bm[(size_t)u * (size_t)wpr + (size_t)(w >> 5)], 1u << (w & 31));
    }
}

hipError_t launch_bitmap_set(const int32_t* src, const int32_t* col, int64_t nnz, int32_t wpr, uint32_t* bitmap,
                             hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(bitmap_set_kernel, dim3(grid_for(nnz, 256)), dim3(256), 0, s, src, col, nnz, wpr, bitmap);
    return hipGetLastError();
}

}  // namespace dm
