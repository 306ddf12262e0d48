"""ctypes binding over libdmotif.so (the C ABI declared in include/dmotif.h).

Argument marshalling only: every step of the enumeration runs in the HIP
library.  PyTorch is used for streams and for device memory handed back to
the caller (``Result.to_torch``).  Method names follow the C entry points:

=======================  ==========================
Python                   C ABI
=======================  ==========================
``Context(...)``         ``dm_context_create``
``DataGraph(...)``       ``dm_datagraph_build``
``DataGraph.enumerate``  ``dm_enumerate``
``DataGraph.enumerate_batch``  ``dm_enumerate_batch``
``DataGraph.estimate``   ``dm_estimate``
``Server.submit/wait``   ``dm_server_submit/_wait``
``plan(...)``            ``dm_plan``
=======================  ==========================
"""
from __future__ import annotations

import ctypes as C
import os
import threading
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmotif.so")

DM_OK = 0
STATUS = {0: "DM_OK", -1: "DM_ERR_INVALID_ARG", -2: "DM_ERR_VERTEX_RANGE", -3: "DM_ERR_PATTERN_DISCONNECTED",
          -4: "DM_ERR_PATTERN_SELF_LOOP", -5: "DM_ERR_OUT_OF_MEMORY", -6: "DM_ERR_BUDGET_EXCEEDED",
          -7: "DM_ERR_DEVICE", -8: "DM_ERR_CANCELLED", -9: "DM_ERR_BUSY", -10: "DM_ERR_TIMEOUT",
          -11: "DM_ERR_INTERNAL", -12: "DM_ERR_UNSUPPORTED"}

MOTIF_M3, MOTIF_M4, MOTIF_M5, MOTIF_M6 = 1 << 0, 1 << 1, 1 << 2, 1 << 3
MOTIF_C4, MOTIF_C6, MOTIF_C12 = 1 << 4, 1 << 5, 1 << 6
MOTIF_M4_1, MOTIF_M6_2O, MOTIF_M18_O_6, MOTIF_M7 = 1 << 7, 1 << 8, 1 << 9, 1 << 10
MOTIF_ALL, MOTIF_AUTO, MOTIF_M2_ONLY = 0x7FF, 0, 0x80000000
MOTIF_NAMES = ["M2", "M3", "M4", "M5", "M6", "M4-O", "M6-O", "M12-O", "M4-1", "M6-2O", "M18-O-6", "M7"]
MAX_PATTERN_VERTICES = 128

OUT_TABLE, OUT_COUNT_HASH = 0, 1


class DMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GraphDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_edges", C.c_int64), ("edges", C.POINTER(C.c_int32))]


# GraphDesc as a numpy record, for building the descriptor array of a batch
# in one step (per-pattern ctypes objects cost microseconds each)
_DESC_DT = np.dtype({"names": ["n_vertices", "n_edges", "edges"], "formats": [np.int32, np.int64, np.uint64],
                     "offsets": [GraphDesc.n_vertices.offset, GraphDesc.n_edges.offset, GraphDesc.edges.offset],
                     "itemsize": C.sizeof(GraphDesc)})


_I32 = np.dtype(np.int32)


def _edge_array(edges) -> np.ndarray:
    if type(edges) is np.ndarray and edges.dtype == _I32 and edges.ndim == 2 and edges.flags.c_contiguous:
        return edges
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


def _desc_array(patterns):
    """(descriptor array, the one edge array it points into) for a list of
    (n, edges): the edge lists are packed back to back, so every pointer is
    the block's address plus an offset."""
    arrs = [_edge_array(e) for _, e in patterns]
    k = len(arrs)
    m = np.fromiter((a.shape[0] for a in arrs), dtype=np.int64, count=k)
    block = np.concatenate(arrs) if k else np.zeros((0, 2), dtype=np.int32)
    d = np.empty(k, dtype=_DESC_DT)
    d["n_vertices"] = np.fromiter((int(n) for n, _ in patterns), dtype=np.int32, count=k)
    d["n_edges"] = m
    start = np.zeros(k, dtype=np.uint64)
    if k > 1:
        start[1:] = np.cumsum(m[:-1]).astype(np.uint64) * np.uint64(8)
    d["edges"] = np.uint64(block.__array_interface__["data"][0]) + start
    return d, block


class PlanOpts(C.Structure):
    _fields_ = [("motif_mask", C.c_uint32), ("block_threads", C.c_int32), ("output_mode", C.c_int32),
                ("sync_each_step", C.c_int32), ("mem_budget", C.c_int64), ("profile", C.c_int32),
                ("induced", C.c_int32), ("initial_rows", C.c_int64), ("root_begin", C.c_int32),
                ("root_end", C.c_int32), ("score", C.c_int32), ("result_mb", C.c_int32),
                ("wait_limit_us", C.c_int32)]


class DataGraphInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_directed_edges", C.c_int64), ("max_degree", C.c_int32),
                ("has_bitmap", C.c_int32), ("motif_mask", C.c_uint32), ("motif_rows", C.c_int64 * 12),
                ("build_ms", C.c_double)]


class RunStats(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("retries", C.c_int32), ("chunks", C.c_int32), ("reserved", C.c_int32),
                ("step_rows", C.c_int64 * MAX_PATTERN_VERTICES), ("plan_ms", C.c_double),
                ("device_ms", C.c_double), ("bytes_moved", C.c_int64), ("join_launches", C.c_int32),
                ("sort_launches", C.c_int32), ("join_ms", C.c_double), ("sort_ms", C.c_double),
                ("join_bytes", C.c_int64), ("sort_bytes", C.c_int64)]


class BatchTuning(C.Structure):
    """``dm_batch_tuning``: launch shape of the batched form."""
    _fields_ = [("block_threads", C.c_int32), ("grid", C.c_int32), ("backoff", C.c_int32),
                ("reserved", C.c_int32), ("ms", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("max_batch", C.c_int32), ("mem_budget", C.c_int64),
                ("max_queue", C.c_int32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """``dm_allocator``: device-memory callbacks of a context."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


_lock = threading.Lock()
_LIB = None

# Every symbol include/dmotif.h declares (checked by the CPU test suite).
EXPORTS = [
    "dm_version", "dm_last_error", "dm_context_create", "dm_context_destroy", "dm_context_cancel",
    "dm_datagraph_build",
    "dm_datagraph_free", "dm_datagraph_save", "dm_datagraph_load", "dm_datagraph_set_costs",
    "dm_result_device_costs", "dm_result_copy_costs", "dm_autotune_motifs", "dm_autotune_batch", "dm_datagraph_query", "dm_datagraph_copy_csr", "dm_datagraph_copy_motif", "dm_plan",
    "dm_estimate", "dm_enumerate", "dm_enumerate_noalloc", "dm_enumerate_batch", "dm_result_rows",
    "dm_result_total",
    "dm_result_width", "dm_result_device_data", "dm_result_hash", "dm_result_copy_to_host",
    "dm_result_copy_to_device", "dm_result_stats", "dm_result_free", "dm_result_summaries",
    "dm_result_free_many", "dm_server_start", "dm_server_submit", "dm_server_wait", "dm_server_wait_any", "dm_server_stop",
]


def lib() -> C.CDLL:
    """Load libdmotif.so.  Raises if the HIP library has not been built: there
    is no fallback path."""
    global _LIB
    if _LIB is not None:  # set once, under the lock below
        return _LIB
    with _lock:
        if _LIB is not None:
            return _LIB
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_21287_amd._build`")
        # PyTorch ships its own HIP runtime with the same soname as the system
        # one (libamdhip64.so.7).  Loading torch first makes the library bind to
        # that already-loaded runtime, so the process holds a single HIP/HSA
        # instance and streams/pointers are shared with torch.
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32p = C.c_void_p, C.POINTER(C.c_int32)
        sig = {
            "dm_version": (C.c_char_p, []),
            "dm_last_error": (C.c_char_p, []),
            "dm_context_create": (C.c_int, [C.c_int32, vp, C.POINTER(Allocator), C.POINTER(vp)]),
            "dm_context_destroy": (None, [vp]),
            "dm_context_cancel": (C.c_int, [vp, C.c_int32]),
            "dm_datagraph_build": (C.c_int, [vp, C.POINTER(GraphDesc), C.c_uint32, C.POINTER(vp)]),
            "dm_datagraph_free": (C.c_int, [vp]),
            "dm_datagraph_save": (C.c_int, [vp, C.c_char_p]),
            "dm_autotune_batch": (C.c_int, [vp, C.c_int32, C.POINTER(GraphDesc), C.c_int32,
                                            C.POINTER(BatchTuning), C.POINTER(BatchTuning), C.c_int32,
                                            C.POINTER(C.c_int32)]),
            "dm_autotune_motifs": (C.c_int, [vp, C.POINTER(GraphDesc), C.c_int32, C.POINTER(GraphDesc),
                                             C.POINTER(C.c_uint32), C.c_int32, C.c_int32, C.POINTER(C.c_uint32),
                                             C.POINTER(C.c_double)]),
            "dm_datagraph_set_costs": (C.c_int, [vp, C.POINTER(C.c_uint32), C.c_int64, i32p,
                                                 C.POINTER(C.c_uint32)]),
            "dm_result_device_costs": (vp, [vp]),
            "dm_result_copy_costs": (C.c_int, [vp, C.POINTER(C.c_uint64), C.c_int64]),
            "dm_datagraph_load": (C.c_int, [vp, C.c_char_p, C.POINTER(vp)]),
            "dm_datagraph_query": (C.c_int, [vp, C.POINTER(DataGraphInfo)]),
            "dm_datagraph_copy_csr": (C.c_int, [vp, i32p, i32p]),
            "dm_datagraph_copy_motif": (C.c_int, [vp, C.c_int32, C.c_int32, i32p, C.c_int64,
                                                  C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
            "dm_plan": (C.c_int, [C.POINTER(GraphDesc), C.c_uint32, i32p, C.c_int32, i32p]),
            "dm_estimate": (C.c_int, [vp, C.POINTER(GraphDesc), C.POINTER(PlanOpts), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]),
            "dm_enumerate": (C.c_int, [vp, C.POINTER(GraphDesc), C.c_int64, C.POINTER(PlanOpts), C.POINTER(vp)]),
            "dm_enumerate_noalloc": (C.c_int, [vp, C.POINTER(GraphDesc), C.c_int64, C.POINTER(PlanOpts), vp,
                                               C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                               C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
            "dm_enumerate_batch": (C.c_int, [vp, C.c_int32, C.POINTER(GraphDesc), C.POINTER(C.c_int64),
                                             C.POINTER(PlanOpts), C.POINTER(vp)]),
            "dm_result_rows": (C.c_int64, [vp]),
            "dm_result_total": (C.c_int64, [vp]),
            "dm_result_width": (C.c_int32, [vp]),
            "dm_result_device_data": (vp, [vp]),
            "dm_result_hash": (C.c_int, [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
            "dm_result_copy_to_host": (C.c_int, [vp, i32p, C.c_int64]),
            "dm_result_copy_to_device": (C.c_int, [vp, vp, C.c_int64, vp]),
            "dm_result_stats": (C.c_int, [vp, C.POINTER(RunStats)]),
            "dm_result_free": (None, [vp]),
            "dm_result_summaries": (C.c_int, [vp, C.c_int32, vp]),
            "dm_result_free_many": (None, [vp, C.c_int32]),
            "dm_server_start": (C.c_int, [vp, C.POINTER(ServerOpts), C.POINTER(vp)]),
            "dm_server_submit": (C.c_int, [vp, C.POINTER(GraphDesc), C.c_int64, C.POINTER(C.c_uint64)]),
            "dm_server_wait": (C.c_int, [vp, C.c_uint64, C.c_int32, C.POINTER(vp)]),
            "dm_server_wait_any": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_uint64), C.POINTER(vp),
                                             C.POINTER(C.c_int32)]),
            "dm_server_stop": (C.c_int, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
        return L


def _check(code: int):
    if code != DM_OK:
        msg = lib().dm_last_error()
        raise DMError(code, msg.decode() if msg else "")


class _Graph:
    """Keeps a GraphDesc and the int32 array it points to alive together."""

    def __init__(self, n: int, edges):
        self.arr = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        self.desc = GraphDesc(int(n), int(self.arr.shape[0]), self.arr.ctypes.data_as(C.POINTER(C.c_int32)))


def _opts(motif_mask=0, block=0, mode=OUT_TABLE, sync_each_step=False, mem_budget=0,
          profile=False, initial_rows=0, root_range=None, induced=False, score=False,
          result_mb=0, wait_limit_us=0) -> PlanOpts:
    rb, re = (0, 0) if root_range is None else (int(root_range[0]), int(root_range[1]))
    return PlanOpts(int(motif_mask) & 0xFFFFFFFF, int(block), int(mode), int(bool(sync_each_step)),
                    int(mem_budget), int(bool(profile)), int(bool(induced)), int(initial_rows), rb, re,
                    int(bool(score)), int(result_mb), int(wait_limit_us))


class ResultSummary(C.Structure):
    _fields_ = [("total", C.c_int64), ("rows", C.c_int64), ("join_ms", C.c_double), ("sort_ms", C.c_double),
                ("join_bytes", C.c_int64), ("sort_bytes", C.c_int64), ("join_launches", C.c_int32),
                ("sort_launches", C.c_int32)]


_SUMMARY_DT = np.dtype({"names": [f[0] for f in ResultSummary._fields_],
                        "formats": [np.int64, np.int64, np.float64, np.float64, np.int64, np.int64, np.int32,
                                    np.int32],
                        "offsets": [getattr(ResultSummary, f[0]).offset for f in ResultSummary._fields_],
                        "itemsize": C.sizeof(ResultSummary)})


def _handles(results) -> np.ndarray:
    h = np.fromiter(((r._h.value or 0) if r._h else 0 for r in results), dtype=np.uint64, count=len(results))
    if len(results) and not h.all():
        raise ValueError("a result was already freed")
    return h


def summarize(results) -> np.ndarray:
    """``dm_result_summaries``: one record (total, rows, join_ms, sort_ms,
    join_bytes, sort_bytes, join_launches, sort_launches) per result, in one
    call."""
    h = _handles(results)
    out = np.zeros(len(results), dtype=_SUMMARY_DT)
    if len(results):
        _check(lib().dm_result_summaries(C.c_void_p(h.ctypes.data), len(results), C.c_void_p(out.ctypes.data)))
    return out


def free_results(results) -> None:
    """``dm_result_free_many``: free every result of the list in one call."""
    live = [r for r in results if r._h]
    if not live:
        return
    h = _handles(live)
    lib().dm_result_free_many(C.c_void_p(h.ctypes.data), len(live))
    for r in live:
        r._h = None


def _torch_stream(device: int):
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    except Exception:
        pass
    return C.c_void_p(0)


class Context:
    """``dm_context_create``: a device plus the HIP stream all work is ordered
    on (default: torch's current stream on that device).

    ``allocator``: optional ``(alloc, free)`` pair of Python callables,
    ``alloc(nbytes, stream) -> int`` (a device pointer, 0 = failure) and
    ``free(ptr, stream)``, through which the library takes every device
    buffer (``dm_allocator``); they may be called from the library's server
    threads."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        L = lib()
        self.device = device
        if stream is None:
            s = _torch_stream(device)
        elif hasattr(stream, "cuda_stream"):
            s = C.c_void_p(stream.cuda_stream)
        else:
            s = C.c_void_p(int(stream))
        self._h = C.c_void_p()
        self._children = weakref.WeakSet()
        self._alloc = None
        if allocator is not None:
            fa, ff = allocator

            def _a(nbytes, stream, _user):
                try:
                    return int(fa(int(nbytes), int(stream or 0)) or 0) or None
                except Exception:
                    return None

            def _f(ptr, stream, _user):
                try:
                    ff(int(ptr or 0), int(stream or 0))
                except Exception:
                    pass

            # the callbacks must outlive the context: keep them on it
            self._alloc = Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
        _check(L.dm_context_create(device, s, C.byref(self._alloc) if self._alloc is not None else None,
                                   C.byref(self._h)))

    def cancel(self, flag: bool = True) -> None:
        """``dm_context_cancel``: set or clear the context's cancel word."""
        _check(lib().dm_context_cancel(self._h, int(bool(flag))))

    @property
    def handle(self):
        return self._h

    def _adopt(self, obj):
        self._children.add(obj)
        return obj

    def close(self):
        if self._h:
            # servers first (they hold results), then results, then data graphs
            kids = list(self._children)
            for kind in (Server, Result, DataGraph):
                for o in kids:
                    if isinstance(o, kind):
                        try:
                            o._release()
                        except Exception:
                            pass
            lib().dm_context_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune_motifs(self, n: int, edges, sample, candidates, reps: int = 3):
        """``dm_autotune_motifs``: the fastest motif set for this data graph on
        a sample of patterns; returns ``(best_mask, {mask: median_ms})``."""
        g = _Graph(n, edges)
        gs = [_Graph(pn, pe) for pn, pe in sample]
        arr = (GraphDesc * len(gs))(*[x.desc for x in gs])
        cand = (C.c_uint32 * len(candidates))(*[int(c) & 0xFFFFFFFF for c in candidates])
        ms = (C.c_double * len(candidates))()
        best = C.c_uint32()
        _check(lib().dm_autotune_motifs(self.handle, C.byref(g.desc), len(gs), arr, cand, len(candidates),
                                        int(reps), C.byref(best), ms))
        return best.value, {int(c) & 0xFFFFFFFF: ms[i] for i, c in enumerate(candidates)}

    def datagraph(self, n: int, edges, motif_mask: int = MOTIF_AUTO) -> "DataGraph":
        return DataGraph(self, n, edges, motif_mask)


class Result:
    """An embedding table on the device (``dm_result``)."""

    def __init__(self, h, ctx: "Context | None" = None):
        self._h = h
        if ctx is not None:
            ctx._adopt(self)

    @property
    def rows(self) -> int:
        return int(lib().dm_result_rows(self._h))

    @property
    def total(self) -> int:
        return int(lib().dm_result_total(self._h))

    @property
    def width(self) -> int:
        return int(lib().dm_result_width(self._h))

    @property
    def device_ptr(self) -> int:
        return int(lib().dm_result_device_data(self._h) or 0)

    def to_numpy(self, max_rows: int | None = None) -> np.ndarray:
        n = self.rows if max_rows is None else min(max_rows, self.rows)
        out = np.empty((n, self.width), dtype=np.int32)
        if n:
            _check(lib().dm_result_copy_to_host(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)), n))
        return out

    def to_torch(self, device: int | None = None):
        """Device-to-device copy into a torch int32 tensor [rows, width]."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        t = torch.empty((self.rows, self.width), dtype=torch.int32, device=dev)
        if self.rows:
            s = torch.cuda.current_stream(dev).cuda_stream
            _check(lib().dm_result_copy_to_device(self._h, C.c_void_p(t.data_ptr()), self.rows, C.c_void_p(s)))
        return t

    def costs(self) -> np.ndarray:
        """Scored runs: the layout cost of every held row (uint64)."""
        out = np.zeros(self.rows, np.uint64)
        if self.rows:
            _check(lib().dm_result_copy_costs(self._h, out.ctypes.data_as(C.POINTER(C.c_uint64)), self.rows))
        return out

    def hash(self) -> tuple[int, int]:
        hs, hx = C.c_uint64(), C.c_uint64()
        _check(lib().dm_result_hash(self._h, C.byref(hs), C.byref(hx)))
        return hs.value, hx.value

    def stats(self) -> dict:
        st = RunStats()
        _check(lib().dm_result_stats(self._h, C.byref(st)))
        n = st.n_steps
        return {"n_steps": n, "retries": st.retries, "chunks": st.chunks,
                "step_rows": [int(x) for x in st.step_rows[:max(n, 1)]], "plan_ms": st.plan_ms,
                "device_ms": st.device_ms, "bytes_moved": int(st.bytes_moved),
                "join_launches": st.join_launches, "sort_launches": st.sort_launches, "join_ms": st.join_ms,
                "sort_ms": st.sort_ms, "join_bytes": int(st.join_bytes), "sort_bytes": int(st.sort_bytes)}

    def timing(self) -> tuple:
        """(join_ms, join_bytes, join_launches, sort_ms, sort_bytes) of ``dm_result_stats``
        without building the full dict (for per-step accounting in timed loops)."""
        st = RunStats()
        _check(lib().dm_result_stats(self._h, C.byref(st)))
        return st.join_ms, st.join_bytes, st.join_launches, st.sort_ms, st.sort_bytes

    def free(self):
        if self._h:
            lib().dm_result_free(self._h)
            self._h = None

    _release = free

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class DataGraph:
    """``dm_datagraph_build``: normalized data graph + motif tables, resident."""

    def __init__(self, ctx: Context, n: int, edges, motif_mask: int = MOTIF_AUTO, _handle=None):
        self.ctx = ctx
        self._h = C.c_void_p()
        if _handle is not None:
            self._h = _handle
        else:
            g = _Graph(n, edges)
            _check(lib().dm_datagraph_build(ctx.handle, C.byref(g.desc), int(motif_mask) & 0xFFFFFFFF,
                                            C.byref(self._h)))
        ctx._adopt(self)

    @classmethod
    def load(cls, ctx: Context, path: str) -> "DataGraph":
        """``dm_datagraph_load``: a database written by :meth:`save`."""
        h = C.c_void_p()
        _check(lib().dm_datagraph_load(ctx.handle, os.fsencode(path), C.byref(h)))
        return cls(ctx, 0, None, _handle=h)

    def set_costs(self, vertex_cost=None, cost_edges=None, edge_cost=None) -> None:
        """``dm_datagraph_set_costs``: integer layout costs per vertex and per
        listed edge (unlisted edges cost 0)."""
        u32p = C.POINTER(C.c_uint32)
        vc = None
        if vertex_cost is not None:
            vc = np.ascontiguousarray(np.asarray(vertex_cost, dtype=np.uint32))
            if len(vc) != self.info()["n_vertices"]:
                raise ValueError("vertex_cost needs one entry per data vertex")
        ce = np.ascontiguousarray(np.asarray(cost_edges if cost_edges is not None else np.zeros((0, 2)),
                                             dtype=np.int32).reshape(-1, 2))
        ec = np.ascontiguousarray(np.asarray(edge_cost if edge_cost is not None else [], dtype=np.uint32))
        if len(ec) != len(ce):
            raise ValueError("edge_cost needs one entry per cost edge")
        _check(lib().dm_datagraph_set_costs(self._h, vc.ctypes.data_as(u32p) if vc is not None else None,
                                            len(ce), ce.ctypes.data_as(C.POINTER(C.c_int32)),
                                            ec.ctypes.data_as(u32p) if len(ec) else None))

    def save(self, path: str) -> None:
        """``dm_datagraph_save``: the CSR and every motif table, to a file."""
        _check(lib().dm_datagraph_save(self._h, os.fsencode(path)))

    def info(self) -> dict:
        i = DataGraphInfo()
        _check(lib().dm_datagraph_query(self._h, C.byref(i)))
        return {"n_vertices": i.n_vertices, "n_directed_edges": i.n_directed_edges,
                "max_degree": i.max_degree, "has_bitmap": bool(i.has_bitmap), "motif_mask": i.motif_mask,
                "motif_rows": {MOTIF_NAMES[m]: int(i.motif_rows[m]) for m in range(len(MOTIF_NAMES))},
                "build_ms": i.build_ms}

    def csr(self):
        info = self.info()
        rp = np.zeros(info["n_vertices"] + 1, np.int32)
        col = np.zeros(max(info["n_directed_edges"], 1), np.int32)
        _check(lib().dm_datagraph_copy_csr(self._h, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                           col.ctypes.data_as(C.POINTER(C.c_int32))))
        return rp, col[:info["n_directed_edges"]]

    def motif_table(self, motif: int, key_pos: int = 0) -> np.ndarray:
        rows, width = C.c_int64(), C.c_int32()
        _check(lib().dm_datagraph_copy_motif(self._h, motif, key_pos, None, 0, C.byref(rows), C.byref(width)))
        out = np.zeros((rows.value, width.value), np.int32)
        if rows.value:
            _check(lib().dm_datagraph_copy_motif(self._h, motif, key_pos,
                                                 out.ctypes.data_as(C.POINTER(C.c_int32)), rows.value,
                                                 C.byref(rows), C.byref(width)))
        return out

    def estimate(self, n: int, edges, motif_mask: int = 0) -> tuple[int, int]:
        g = _Graph(n, edges)
        o = _opts(motif_mask)
        peak, rows = C.c_int64(), C.c_int64()
        _check(lib().dm_estimate(self._h, C.byref(g.desc), C.byref(o), C.byref(peak), C.byref(rows)))
        return peak.value, rows.value

    def enumerate(self, n: int, edges, cap: int = -1, **opts) -> Result:
        g = _Graph(n, edges)
        o = _opts(**opts)
        h = C.c_void_p()
        _check(lib().dm_enumerate(self._h, C.byref(g.desc), int(cap), C.byref(o), C.byref(h)))
        return Result(h, self.ctx)

    def enumerate_noalloc(self, n: int, edges, out_ptr: int, out_rows_cap: int, cap: int = -1,
                          **opts) -> tuple[int, int, tuple[int, int]]:
        """``dm_enumerate_noalloc``: the sorted rows into the caller's device
        buffer at ``out_ptr`` (``out_rows_cap`` rows of ``n`` int32), with no
        device allocation.  Returns ``(rows, total, (hash_sum, hash_xor))``."""
        g = _Graph(n, edges)
        o = _opts(**opts)
        rows, total = C.c_int64(), C.c_int64()
        hs, hx = C.c_uint64(), C.c_uint64()
        _check(lib().dm_enumerate_noalloc(self._h, C.byref(g.desc), int(cap), C.byref(o),
                                          C.c_void_p(int(out_ptr) or None), int(out_rows_cap), C.byref(rows),
                                          C.byref(total), C.byref(hs), C.byref(hx)))
        return rows.value, total.value, (hs.value, hx.value)

    def enumerate_batch(self, patterns, caps=None, **opts) -> list[Result]:
        descs, keep = _desc_array(patterns)
        n = len(descs)
        capv = None
        if caps is not None:
            capv = np.ascontiguousarray(np.asarray(caps, dtype=np.int64))
            if capv.shape != (n,):
                raise ValueError("caps must give one value per pattern")
        outs = np.zeros(max(n, 1), dtype=np.uint64)
        o = _opts(**opts)
        _check(lib().dm_enumerate_batch(
            self._h, n, C.cast(descs.ctypes.data, C.POINTER(GraphDesc)) if n else None,
            None if capv is None else C.cast(capv.ctypes.data, C.POINTER(C.c_int64)), C.byref(o),
            C.cast(outs.ctypes.data, C.POINTER(C.c_void_p))))
        del keep  # the call copied the patterns
        return [Result(C.c_void_p(int(h)), self.ctx) for h in outs[:n].tolist()]

    def autotune_batch(self, patterns, reps: int = 3) -> tuple[dict, list[dict]]:
        """``dm_autotune_batch``: time the batched call on `patterns` for each
        launch shape and keep the fastest on this data graph; returns (best,
        tried) as dicts of block_threads, grid, backoff, ms."""
        descs, keep = _desc_array(patterns)
        n = len(descs)
        best = BatchTuning()
        tried = (BatchTuning * 64)()
        nt = C.c_int32()
        _check(lib().dm_autotune_batch(self._h, n, C.cast(descs.ctypes.data, C.POINTER(GraphDesc)) if n else None,
                                       int(reps), C.byref(best), tried, 64, C.byref(nt)))
        del keep

        def as_dict(t):
            return {"block_threads": t.block_threads, "grid": t.grid, "backoff": t.backoff, "ms": t.ms}

        return as_dict(best), [as_dict(tried[i]) for i in range(min(nt.value, 64))]

    def free(self):
        if self._h:
            _check(lib().dm_datagraph_free(self._h))
            self._h = C.c_void_p()

    _release = free

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """``dm_server_*``: continuous batching over one resident data graph."""

    def __init__(self, dg: DataGraph, n_streams: int = 2, max_batch: int = 64, mem_budget: int = 0,
                 max_queue: int = 0):
        self.dg = dg
        o = ServerOpts(n_streams, max_batch, mem_budget, max_queue)
        self._h = C.c_void_p()
        _check(lib().dm_server_start(dg._h, C.byref(o), C.byref(self._h)))
        dg.ctx._adopt(self)

    def submit(self, n: int, edges, cap: int = -1) -> int:
        g = _Graph(n, edges)
        t = C.c_uint64()
        _check(lib().dm_server_submit(self._h, C.byref(g.desc), int(cap), C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> Result:
        h = C.c_void_p()
        _check(lib().dm_server_wait(self._h, C.c_uint64(ticket), int(timeout_ms), C.byref(h)))
        return Result(h, self.dg.ctx)

    def wait_any(self, timeout_ms: int = -1):
        """``dm_server_wait_any``: (ticket, Result or None, status) of the next
        query to finish; status is the query's own code (0 = OK)."""
        h = C.c_void_p()
        t = C.c_uint64()
        st = C.c_int32()
        _check(lib().dm_server_wait_any(self._h, int(timeout_ms), C.byref(t), C.byref(h), C.byref(st)))
        return t.value, (Result(h, self.dg.ctx) if st.value == 0 else None), st.value

    def stop(self):
        if self._h:
            _check(lib().dm_server_stop(self._h))
            self._h = C.c_void_p()

    _release = stop

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def plan(n: int, edges, motif_mask: int = MOTIF_ALL) -> dict:
    """``dm_plan``: the host decomposition of a pattern (no device needed)."""
    g = _Graph(n, edges)
    need = C.c_int32()
    rc = lib().dm_plan(C.byref(g.desc), int(motif_mask) & 0xFFFFFFFF, None, 0, C.byref(need))
    if need.value <= 0:
        _check(rc)
    buf = np.zeros(need.value, np.int32)
    _check(lib().dm_plan(C.byref(g.desc), int(motif_mask) & 0xFFFFFFFF,
                         buf.ctypes.data_as(C.POINTER(C.c_int32)), need.value, C.byref(need)))
    b = buf.tolist()
    k, ns = b[0], b[1]
    col_of = b[2:2 + k]
    i = 2 + k
    steps = []
    for _ in range(ns):
        st = {"motif": b[i], "key_pos": b[i + 1], "key_col": b[i + 2], "c_in": b[i + 3]}
        i += 4
        nn = b[i]; st["new_pos"] = b[i + 1:i + 1 + nn]; i += 1 + nn
        ne = b[i]; st["eq"] = [(b[i + 1 + 2 * j], b[i + 2 + 2 * j]) for j in range(ne)]; i += 1 + 2 * ne
        nd = b[i]; st["edges"] = [(b[i + 1 + 2 * j], b[i + 2 + 2 * j]) for j in range(nd)]; i += 1 + 2 * nd
        sl = b[i]; st["slice"] = b[i + 1:i + 1 + sl]; i += 1 + sl
        steps.append(st)
    return {"k": k, "col_of": col_of, "steps": steps}
