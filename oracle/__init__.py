"""CPU oracle for subgraph-embedding enumeration (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (the HIP library and its Python binding) never imports, links or calls
it, and the oracle imports nothing from the product package.

What it computes is the definition of the paper's Sec. III-A restricted to
edge preservation (non-induced embeddings): every injective
``f: V_p -> V_d`` with ``{f(u), f(v)} in E_d`` for each pattern edge, as a
lexicographically sorted ``int32`` table with column ``j`` = ``f(j)``.  See
``oracle.c`` for the method and the return codes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, INVALID, RANGE, DISCONNECTED, SELF_LOOP, NOMEM, DUPLICATE = 0, -1, -2, -3, -4, -5, -9

_lock = threading.Lock()
_libs: dict[str, C.CDLL] = {}


def build(out: str = LIB, mutant: int = 0, force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into a shared library (seconds)."""
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", f"-DORACLE_MUTANT={mutant}", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def load(path: str = LIB) -> C.CDLL:
    with _lock:
        if path in _libs:
            return _libs[path]
        if path == LIB and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(LIB)
        lib = C.CDLL(path)
        i32p = C.POINTER(C.c_int32)
        lib.oracle_normalize.restype = C.c_int64
        lib.oracle_normalize.argtypes = [C.c_int32, C.c_int64, i32p, i32p, i32p]
        lib.oracle_enumerate.restype = C.c_int
        lib.oracle_enumerate.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                         C.c_int64, C.POINTER(i32p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]
        lib.oracle_enumerate_range.restype = C.c_int
        lib.oracle_enumerate_range.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                               C.c_int64, C.c_int32, C.c_int32, C.POINTER(i32p),
                                               C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.oracle_count_hash.restype = C.c_int
        lib.oracle_count_hash.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                          C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                          C.POINTER(C.c_uint64)]
        lib.oracle_enumerate_ex.restype = C.c_int
        lib.oracle_enumerate_ex.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                            C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.POINTER(i32p),
                                            C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        lib.oracle_count_hash_range.restype = C.c_int
        lib.oracle_count_hash_range.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                                C.c_int32, C.c_int32, C.POINTER(C.c_int64),
                                                C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        lib.oracle_count_hash_ex.restype = C.c_int
        lib.oracle_count_hash_ex.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                             C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                             C.POINTER(C.c_uint64)]
        u32p, u64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        lib.oracle_enumerate_scored.restype = C.c_int
        lib.oracle_enumerate_scored.argtypes = [C.c_int32, C.c_int64, i32p, C.c_int32, C.c_int64, i32p,
                                                u32p, C.c_int64, i32p, u32p, C.c_int64, C.c_int32,
                                                C.POINTER(i32p), C.POINTER(u64p), C.POINTER(C.c_int64),
                                                C.POINTER(C.c_int64)]
        lib.oracle_row_hash.restype = C.c_uint64
        lib.oracle_row_hash.argtypes = [i32p, C.c_int32]
        lib.oracle_mix64.restype = C.c_uint64
        lib.oracle_mix64.argtypes = [C.c_uint64]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [C.c_void_p]
        lib.oracle_mutant_id.restype = C.c_int
        _libs[path] = lib
        return lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _edges(e) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def normalize(n: int, edges, lib: C.CDLL | None = None):
    """Sorted, duplicate-free, loop-free adjacency (CSR) of an undirected graph."""
    lib = lib or load()
    e = _edges(edges)
    row_ptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(2 * len(e), 1), np.int32)
    nnz = lib.oracle_normalize(n, len(e), _p(e), _p(row_ptr), _p(col))
    if nnz < 0:
        raise OracleError(int(nnz))
    return row_ptr, col[:nnz].copy()


def enumerate_embeddings(n_d: int, edges_d, n_p: int, edges_p, cap: int = -1,
                         lib: C.CDLL | None = None, root_range=None, induced: bool = False):
    """Return ``(rows[int32, n x n_p], total)``: the lexicographically first
    ``cap`` embeddings (all when ``cap < 0``) and the full count; with
    ``root_range=(lo, hi)`` only embeddings with ``f(0)`` in ``[lo, hi)``;
    ``induced=True`` keeps only induced embeddings."""
    lib = lib or load()
    ed, ep = _edges(edges_d), _edges(edges_p)
    rows = C.POINTER(C.c_int32)()
    n_rows, total = C.c_int64(0), C.c_int64(0)
    if induced:
        lo, hi = root_range if root_range is not None else (0, n_d)
        rc = lib.oracle_enumerate_ex(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep), cap, int(lo), int(hi), 1,
                                     C.byref(rows), C.byref(n_rows), C.byref(total))
    elif root_range is None:
        rc = lib.oracle_enumerate(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep), cap,
                                  C.byref(rows), C.byref(n_rows), C.byref(total))
    else:
        rc = lib.oracle_enumerate_range(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep), cap,
                                        int(root_range[0]), int(root_range[1]),
                                        C.byref(rows), C.byref(n_rows), C.byref(total))
    if rc != 0:
        raise OracleError(rc)
    try:
        nr = n_rows.value
        if nr:
            out = np.ctypeslib.as_array(rows, shape=(nr * n_p,)).reshape(nr, n_p).copy()
        else:
            out = np.zeros((0, n_p), np.int32)
    finally:
        if rows:
            lib.oracle_free(C.cast(rows, C.c_void_p))
    return out, total.value


def enumerate_scored(n_d: int, edges_d, n_p: int, edges_p, vertex_cost=None, cost_edges=None, edge_cost=None,
                     top_k: int = -1, induced: bool = False, lib: C.CDLL | None = None):
    """Layout scoring: ``(rows, costs, total)`` with rows ordered by (cost,
    row) ascending, the first ``top_k`` kept (all when negative).  Costs are
    non-negative integers per data vertex and per listed data edge."""
    lib = lib or load()
    ed, ep = _edges(edges_d), _edges(edges_p)
    vc = None
    if vertex_cost is not None:
        vc = np.ascontiguousarray(np.asarray(vertex_cost, dtype=np.uint32))
        assert len(vc) == n_d
    ce = _edges(cost_edges if cost_edges is not None else np.zeros((0, 2), np.int32))
    ec = np.ascontiguousarray(np.asarray(edge_cost if edge_cost is not None else [], dtype=np.uint32))
    assert len(ec) == len(ce)
    rows = C.POINTER(C.c_int32)()
    costs = C.POINTER(C.c_uint64)()
    n_rows, total = C.c_int64(0), C.c_int64(0)
    u32p = C.POINTER(C.c_uint32)
    rc = lib.oracle_enumerate_scored(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep),
                                     vc.ctypes.data_as(u32p) if vc is not None else None,
                                     len(ce), _p(ce), ec.ctypes.data_as(u32p) if len(ec) else None,
                                     int(top_k), int(bool(induced)),
                                     C.byref(rows), C.byref(costs), C.byref(n_rows), C.byref(total))
    if rc != 0:
        raise OracleError(rc)
    try:
        nr = n_rows.value
        if nr:
            out = np.ctypeslib.as_array(rows, shape=(nr * n_p,)).reshape(nr, n_p).copy()
            cst = np.ctypeslib.as_array(costs, shape=(nr,)).copy()
        else:
            out, cst = np.zeros((0, n_p), np.int32), np.zeros(0, np.uint64)
    finally:
        if rows:
            lib.oracle_free(C.cast(rows, C.c_void_p))
        if costs:
            lib.oracle_free(C.cast(costs, C.c_void_p))
    return out, cst, total.value


def count_hash(n_d: int, edges_d, n_p: int, edges_p, lib: C.CDLL | None = None, induced: bool = False):
    """Streaming ``(count, hash_sum, hash_xor)`` without storing rows."""
    lib = lib or load()
    ed, ep = _edges(edges_d), _edges(edges_p)
    cnt, hs, hx = C.c_int64(0), C.c_uint64(0), C.c_uint64(0)
    rc = lib.oracle_count_hash_ex(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep), int(bool(induced)),
                                  C.byref(cnt), C.byref(hs), C.byref(hx))
    if rc != 0:
        raise OracleError(rc)
    return cnt.value, hs.value, hx.value


def count_hash_range(n_d: int, edges_d, n_p: int, edges_p, root_range, lib: C.CDLL | None = None):
    """``count_hash`` restricted to embeddings with ``f(0)`` in ``[lo, hi)``."""
    lib = lib or load()
    ed, ep = _edges(edges_d), _edges(edges_p)
    cnt, hs, hx = C.c_int64(0), C.c_uint64(0), C.c_uint64(0)
    rc = lib.oracle_count_hash_range(n_d, len(ed), _p(ed), n_p, len(ep), _p(ep), int(root_range[0]),
                                     int(root_range[1]), C.byref(cnt), C.byref(hs), C.byref(hx))
    if rc != 0:
        raise OracleError(rc)
    return cnt.value, hs.value, hx.value


def count_hash_threads(n_d: int, edges_d, n_p: int, edges_p, threads: int, root_range=None,
                       lib: C.CDLL | None = None):
    """``count_hash`` (over ``root_range``, default every root) with the roots
    split into ``threads`` contiguous ranges run on host threads (the C code
    releases the interpreter lock); counts and sums add, hashes XOR."""
    from concurrent.futures import ThreadPoolExecutor
    lib = lib or load()
    lo, hi = root_range if root_range is not None else (0, n_d)
    pieces = max(1, min(threads * 8, hi - lo))
    cuts = np.linspace(lo, hi, pieces + 1).astype(np.int64)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        parts = list(ex.map(lambda i: count_hash_range(n_d, edges_d, n_p, edges_p,
                                                       (int(cuts[i]), int(cuts[i + 1])), lib),
                            range(pieces)))
    c = sum(p[0] for p in parts)
    hs = sum(p[1] for p in parts) % (1 << 64)
    hx = 0
    for p in parts:
        hx ^= p[2]
    return c, hs, hx


def row_hash(row, lib: C.CDLL | None = None) -> int:
    lib = lib or load()
    r = np.ascontiguousarray(np.asarray(row, dtype=np.int32))
    return int(lib.oracle_row_hash(_p(r), len(r)))


def mix64(x: int, lib: C.CDLL | None = None) -> int:
    lib = lib or load()
    return int(lib.oracle_mix64(C.c_uint64(x & (2**64 - 1))))
