// The allocation-free entry point: dm_enumerate with every intermediate
// buffer (the ping-pong tables, look-back words, tickets, control block, the
// sort's segment lists and index scratch) in one fixed device array compiled
// into the library, and the sorted table written to the caller's buffer.
//
// Each device holds its own copy of `scratch` for the life of the process.
// Host code never uses the array's name as an address: the device address of
// a device's copy is taken once per device with hipGetSymbolAddress, with
// that device current, and only that pointer reaches kernels and copies.
#include <cstring>
#include <mutex>
#include <string>

#include "runtime.hpp"

namespace dm {
namespace {

constexpr size_t kScratchBytes = (size_t)DM_NOALLOC_SCRATCH_MB << 20;
// look-back words: a step of r rows uses r / 64 + 2 of them at most
constexpr int64_t kStatusWords = (int64_t)1 << 16;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// One device's share: the address of its copy of the array, the look-back
// epoch that persists across calls (so words left by earlier calls never
// read as ready), and the host-side mirrors the readbacks land in.
struct DeviceScratch {
    std::mutex mu;  // calls on one device share the array: one at a time
    bool ready = false;
    char* ptr = nullptr;
    uint32_t epoch = 0;
    Control host_ctrl;
    SortJob host_job;
};
DeviceScratch g_dev[kMaxDevices];

// Fixed part of the layout (independent of the data graph and pattern):
// control block, sort job, one ticket per epoch, the look-back words.
struct FixedLayout {
    size_t ctrl, job, tickets, status, end;
};
constexpr FixedLayout fixed_layout() {
    FixedLayout f{};
    size_t off = 0;
    f.ctrl = off;
    off = (off + sizeof(Control) + 255) & ~(size_t)255;
    f.job = off;
    off = (off + sizeof(SortJob) + 255) & ~(size_t)255;
    f.tickets = off;
    off = (off + sizeof(uint64_t) * kEpochs + 255) & ~(size_t)255;
    f.status = off;
    off = (off + sizeof(uint64_t) * (size_t)kStatusWords + 255) & ~(size_t)255;
    f.end = off;
    return f;
}
constexpr FixedLayout kFixed = fixed_layout();
static_assert(kFixed.end + ((size_t)1 << 20) < kScratchBytes, "scratch too small for its fixed part");

// First call on a device (that device current): the device address of its
// copy of the array, and cleared tickets and look-back words.
dm_status setup(DeviceScratch& d, hipStream_t s) {
    if (d.ready) return DM_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(DM_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    d.ptr = (char*)p;
    DM_HIP(launch_fill_u64((uint64_t*)(d.ptr + kFixed.tickets), 0, kEpochs, s));
    DM_HIP(launch_fill_u64((uint64_t*)(d.ptr + kFixed.status), 0, kStatusWords, s));
    d.epoch = 0;
    d.ready = true;
    return DM_OK;
}

// A workspace over the device's scratch for a data graph of nv vertices and
// a pattern of k vertices: the variable part holds the segment lists, then
// the sort's index scratch and the two tables at the largest row capacity
// that fits.
dm_status scratch_workspace(DeviceScratch& d, dm_context* ctx, int32_t nv, int k, Workspace* ws) {
    Workspace& w = *ws;
    w.ctx = ctx;
    w.stream = ctx->stream;
    w.fixed = true;
    w.ctrl_d = (Control*)(d.ptr + kFixed.ctrl);
    w.ctrl_h = &d.host_ctrl;
    w.job_d = (SortJob*)(d.ptr + kFixed.job);
    w.job_h = &d.host_job;
    w.tickets = (uint64_t*)(d.ptr + kFixed.tickets);
    w.status = (uint64_t*)(d.ptr + kFixed.status);
    w.status_cap = kStatusWords;
    w.epoch = d.epoch;
    size_t off = kFixed.end;
    const int64_t spill = (int64_t)nv + 1;
    w.spill = (SegRef*)(d.ptr + off);
    w.spill_cap = spill;
    off += sizeof(SegRef) * 2 * (size_t)spill;
    w.spill_bits = (uint32_t*)(d.ptr + off);
    off = align256(off + sizeof(uint32_t) * (size_t)spill);
    if (off + 4096 > kScratchBytes) return fail(DM_ERR_BUDGET_EXCEEDED, "data graph too large for the fixed scratch");
    // the sort's epoch words: this layout moves with nv, so they start clear on every call
    DM_HIP(launch_fill_i32((int32_t*)w.spill_bits, 0, spill, w.stream));
    // rows r: index scratch (2r + 2) uint32 + two tables of r x k int32,
    // and r / 64 + 2 look-back words per step
    const size_t left = kScratchBytes - off - 3 * 256;
    int64_t r = (int64_t)((left - 8) / (8 * (size_t)k + 8));
    r = std::min<int64_t>(r, (kStatusWords - 2) * 64);
    r &= ~(int64_t)63;
    if (r < 64) return fail(DM_ERR_BUDGET_EXCEEDED, "pattern too wide for the fixed scratch");
    w.sort_scratch = (uint32_t*)(d.ptr + off);
    w.sort_scratch_elems = 2 * r + 2;
    off = align256(off + sizeof(uint32_t) * (size_t)(2 * r + 2));
    for (int b = 0; b < 2; b++) {
        w.buf[b] = (int32_t*)(d.ptr + off);
        w.buf_elems[b] = r * k;
        off = align256(off + sizeof(int32_t) * (size_t)(r * k));
    }
    if (off > kScratchBytes) return fail(DM_ERR_INTERNAL, "fixed scratch layout overruns the array");
    return DM_OK;
}

}  // namespace
}  // namespace dm

using namespace dm;

extern "C" dm_status dm_enumerate_noalloc(dm_datagraph* dg, const dm_graph_desc* gp, int64_t max_embeddings,
                                          const dm_plan_opts* opts, int32_t* out, int64_t out_rows_cap,
                                          int64_t* rows, int64_t* total, uint64_t* hash_sum, uint64_t* hash_xor) {
    if (!dg || !gp || !rows || !total) return fail(DM_ERR_INVALID_ARG, "NULL argument");
    const int32_t mode = opts ? opts->output_mode : DM_OUT_TABLE;
    if (mode != DM_OUT_TABLE && mode != DM_OUT_COUNT_HASH) return fail(DM_ERR_INVALID_ARG, "bad output mode");
    if (opts && (opts->score || opts->profile))
        return fail(DM_ERR_UNSUPPORTED, "layout scoring and per-launch profiling need allocations");
    if (mode == DM_OUT_TABLE && out_rows_cap > 0 && !out) return fail(DM_ERR_INVALID_ARG, "out is NULL with rows");
    if (out_rows_cap < 0) return fail(DM_ERR_INVALID_ARG, "negative out_rows_cap");
    if (opts && opts->block_threads != 0 && opts->block_threads != 64 && opts->block_threads != 128 &&
        opts->block_threads != 256)
        return fail(DM_ERR_INVALID_ARG, "block_threads must be 0, 64, 128 or 256");
    dm_context* ctx = dg->ctx;
    if (ctx->device < 0 || ctx->device >= kMaxDevices) return fail(DM_ERR_UNSUPPORTED, "device index too large");
    if (__atomic_load_n(ctx->cancel, __ATOMIC_SEQ_CST)) return fail(DM_ERR_CANCELLED, "context is cancelled");
    DM_HIP(hipSetDevice(ctx->device));

    NormPattern p;
    std::string err;
    dm_status st = normalize_pattern(gp, &p, &err);
    if (st != DM_OK) return fail(st, err);
    if (p.k > dg->n) {
        *rows = 0;
        *total = 0;
        if (hash_sum) *hash_sum = 0;
        if (hash_xor) *hash_xor = 0;
        return DM_OK;
    }
    Plan plan;
    DM_TRY(plan_for(dg, p, opts, &plan));
    RunOptions ro = run_options(opts, max_embeddings);
    ro.profile = false;
    ro.out_buf = out;
    ro.out_buf_rows = out_rows_cap;
    // no destination rows: only the count, without the sort
    if (mode == DM_OUT_TABLE && (!out || out_rows_cap == 0)) ro.sort = false;

    DeviceScratch& d = g_dev[ctx->device];
    std::lock_guard<std::mutex> lock(d.mu);
    DM_TRY(setup(d, ctx->stream));
    Workspace ws;
    DM_TRY(scratch_workspace(d, ctx, dg->n, p.k, &ws));
    RunOutput o;
    st = run_plan(ctx, ws, dg, plan, ro, &o);
    d.epoch = ws.epoch;  // epochs used by this call stay used
    if (st == DM_ERR_BUDGET_EXCEEDED && mode == DM_OUT_TABLE && o.rows > 0) {
        *total = o.rows;  // the rows did not fit the caller's buffer: report how many there are
        return st;
    }
    if (st != DM_OK) return st;
    *total = o.rows;
    *rows = (mode == DM_OUT_TABLE && ro.sort) ? o.sorted_rows : 0;
    if (hash_sum) *hash_sum = o.hsum;
    if (hash_xor) *hash_xor = o.hxor;
    return DM_OK;
}
