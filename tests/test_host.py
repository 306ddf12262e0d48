"""Host-side checks that need no GPU: the C ABI library loads and exports
every declared symbol, pattern validation, and the planner's decomposition
(paper Sec. III-C) executed by a naive CPU table executor against the oracle."""
import re
import os

import numpy as np
import pytest

import oracle
import paper_2508_21287_amd as dm
from paper_2508_21287_amd import workloads as W
import plan_exec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "dmotif.h")).read()
    declared = set(re.findall(r"\b(dm_[a-z_]+)\s*\(", hdr))
    assert declared == set(dm.EXPORTS), declared ^ set(dm.EXPORTS)
    L = dm.lib()
    for name in declared:
        assert getattr(L, name) is not None
    assert L.dm_version().startswith(b"dmotif")


def test_pattern_validation_codes():
    cases = [(2, [[0, 0], [0, 1]], -4), (4, [[0, 1], [2, 3]], -3), (2, [[0, 2]], -2), (0, [], -1),
             (200, [[i, i + 1] for i in range(199)], -12)]
    for n, e, code in cases:
        with pytest.raises(dm.DMError) as ei:
            dm.plan(n, e)
        assert ei.value.code == code, (n, e)


def test_paper_c6_decomposition_with_m4():
    # Sec. III-B: the 6-cycle decomposes into two M4 slices joined on two
    # shared vertices (constraints S0[0]=S1[3] and S0[3]=S1[0]).
    c6 = W.cycle(6)
    pl = dm.plan(c6.n, c6.edges, dm.MOTIF_M4)
    assert len(pl["steps"]) == 2
    s0, s1 = pl["steps"]
    assert s0["motif"] == 2 and s1["motif"] == 2
    shared = set(s0["slice"]) & set(s1["slice"])
    assert len(shared) == 2
    assert len(s1["eq"]) + 1 == 2  # index key + one further key
    ends0 = {s0["slice"][0], s0["slice"][3]}
    ends1 = {s1["slice"][0], s1["slice"][3]}
    assert shared == ends0 == ends1


def _all_patterns():
    pats = [W.path(k) for k in range(1, 8)] + [W.cycle(k) for k in (3, 4, 5, 6, 8, 12)] + [W.star(3)]
    pats += [W.prufer_tree(k, s) for k in (5, 7, 9) for s in range(3)]
    g23, g33 = W.grid(2, 3), W.grid(3, 3)
    pats += [W.Pattern(g23.n, g23.edges, "grid2x3"), W.Pattern(g33.n, g33.edges, "grid3x3")]
    pats += [W.Pattern(4, [[0, 1], [1, 2], [2, 3], [3, 0], [0, 2]], "diamond"),
             W.Pattern(5, [[4, 0], [0, 2], [2, 4], [2, 1], [1, 3]], "tri-tail"),
             W.Pattern(5, [[0, 1], [0, 2], [0, 3], [0, 4], [1, 2], [2, 3], [3, 4], [4, 1]], "wheel4")]
    return pats


@pytest.mark.parametrize("mask", [dm.MOTIF_M2_ONLY, dm.MOTIF_M3, dm.MOTIF_M4, dm.MOTIF_C4 | dm.MOTIF_M4,
                                  dm.MOTIF_ALL], ids=["M2", "M3", "M4", "C4+M4", "all"])
def test_plan_structure(mask):
    for p in _all_patterns():
        pl = dm.plan(p.n, p.edges, mask)
        k = p.n
        assert sorted(pl["col_of"]) == list(range(k))
        assert pl["col_of"][0] == 0  # vertex 0 owns the identity (root) column
        cols = 1
        covered = set()
        edges = {tuple(sorted(e)) for e in p.edges.tolist()}
        pv = {c: v for v, c in enumerate(pl["col_of"])}
        for st in pl["steps"]:
            assert st["c_in"] == cols
            if st["motif"] >= 0:
                if st["motif"] > 0:  # M2 is always allowed; others only when in the mask
                    assert not (mask & dm.MOTIF_M2_ONLY) and (mask >> (st["motif"] - 1)) & 1
                kind, size = plan_exec.MOTIF_SHAPES[st["motif"]]
                sl = st["slice"]
                assert len(sl) == size and len(set(sl)) == size
                placed = [i for i in range(size) if pl["col_of"][sl[i]] < cols]
                assert placed and st["key_pos"] in placed  # slices overlap earlier ones (Sec. III-B)
                me = [tuple(sorted((sl[a], sl[b]))) for a, b in plan_exec.motif_pattern(st["motif"]).edges.tolist()]
                fresh = [e for e in me if e not in covered]
                assert fresh  # every slice covers a new pattern edge
                if kind in ("path", "cycle"):
                    assert len(fresh) == len(me)  # path and cycle slices follow uncovered edges only
                for e in me:
                    assert e in edges  # motif edges land on pattern edges (covered ones repeat a constraint)
                    covered.add(e)
                cols += len(st["new_pos"])
            for a, b in st["edges"]:
                e = tuple(sorted((pv[a], pv[b])))
                assert e in edges and e not in covered
                covered.add(e)
        assert cols == k and covered == edges
        if mask == dm.MOTIF_M2_ONLY:
            # Sec. IV-B: one join per pattern edge (chord joins fused as checks)
            n_joins = sum(1 for st in pl["steps"] if st["motif"] >= 0)
            n_checks = sum(len(st["edges"]) for st in pl["steps"])
            assert n_joins + n_checks == len(edges)


@pytest.mark.parametrize("mask", [dm.MOTIF_M2_ONLY, dm.MOTIF_M4, dm.MOTIF_ALL], ids=["M2", "M4", "all"])
def test_plan_independence_cpu(mask, oracle_lib):
    """Any valid decomposition reaches the same embedding set (Sec. III-C)."""
    graphs = [W.heavy_hex(3, 9), W.grid(4, 5), W.random_gnp(9, 0.4, 11)]
    for g in graphs:
        for p in _all_patterns():
            if p.n > 9:
                continue
            pl = dm.plan(p.n, p.edges, mask)
            got = plan_exec.execute(g, pl)
            want, _ = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
            assert np.array_equal(got, want), (g.name, p.name, mask)
    g, pats = W.config1()
    for p in pats:
        pl = dm.plan(p.n, p.edges, mask)
        want, _ = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
        assert np.array_equal(plan_exec.execute(g, pl), want), p.name


def test_workload_shapes():
    for (R, Cc), (nv, ne, cells) in {(3, 9): (32, 34, 3), (7, 19): (163, 186, 24), (28, 28): (973, 1134, 162),
                                     (40, 40): (1990, 2340, 351), (60, 60): (4485, 5310, 826)}.items():
        g = W.heavy_hex(R, Cc)
        assert (g.n, len(g.edges), W.heavy_hex_cells(R, Cc)) == (nv, ne, cells)
    g, pats = W.config2()
    assert len(pats) == 64 and all(8 <= p.n <= 30 for p in pats)
    g4, pats4 = W.config4(32)
    assert all(4 <= p.n <= 40 for p in pats4)
    # patterns are connected lattice subgraphs with their planted embedding
    for gg, ps in ((g, pats[:16]), (g4, pats4[:16])):
        a = {tuple(e) for e in gg.edges.tolist()} | {tuple(e[::-1]) for e in gg.edges.tolist()}
        for p in ps:
            for u, v in p.edges.tolist():
                assert (int(p.planted[u]), int(p.planted[v])) in a
    # seeds reproduce
    _, again = W.config2()
    assert all(np.array_equal(a.edges, b.edges) for a, b in zip(pats, again))


def test_batch_descriptor_marshalling():
    # the batch call's descriptors are one record array over one packed edge
    # block: every record must read back as the ctypes GraphDesc the C ABI
    # declares, pointing at that pattern's own edges (lists, int64 arrays and
    # empty edge lists included)
    import ctypes as C
    from paper_2508_21287_amd import _binding as B
    _, pats = W.config2(12)
    specs = [(p.n, p.edges) for p in pats]
    specs += [(3, [(0, 1), (1, 2)]), (1, []), (2, np.array([[0, 1]], dtype=np.int64))]
    d, block = B._desc_array(specs)
    assert d.itemsize == C.sizeof(B.GraphDesc)
    descs = (B.GraphDesc * len(specs)).from_address(d.ctypes.data)
    for (n, e), g in zip(specs, descs):
        want = np.asarray(e, dtype=np.int32).reshape(-1, 2)
        assert g.n_vertices == n and g.n_edges == want.shape[0]
        if want.shape[0]:
            got = np.ctypeslib.as_array(g.edges, shape=(2 * want.shape[0],)).reshape(-1, 2)
            assert np.array_equal(got, want)


def test_context_arguments_checked_before_any_device_call():
    import ctypes as C
    from paper_2508_21287_amd import _binding as B
    L = dm.lib()
    h = C.c_void_p()
    # an allocator without a free callback is refused before the device is touched
    bad = B.Allocator(B._ALLOC_FN(lambda n, s, u: None), B._FREE_FN(), None)
    assert L.dm_context_create(0, None, C.byref(bad), C.byref(h)) == -1
    assert b"allocator" in L.dm_last_error()
    assert not h.value
    assert L.dm_context_create(0, None, None, None) == -1
    assert L.dm_context_cancel(None, 1) == -1
