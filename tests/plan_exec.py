"""A naive CPU executor for the planner's decomposition (test harness only).

It runs a plan returned by ``dm_plan`` with plain Python/numpy joins over
motif tables Res(M) taken from the oracle, so that the planner's host logic
(slices, key columns, further keys, new columns, edge checks) can be checked
on the CPU against the oracle's embedding set.  It shares no code with the
HIP path.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2508_21287_amd import workloads as W

MOTIF_SHAPES = {0: ("path", 2), 1: ("path", 3), 2: ("path", 4), 3: ("path", 5), 4: ("path", 6),
                5: ("cycle", 4), 6: ("cycle", 6), 7: ("cycle", 12), 8: ("claw", 4), 9: ("grid2x3", 6),
                10: ("cell18", 18), 11: ("path", 7)}

# heavy-hex cell with pendants: cycle 0-1-3-4-...-12-0, pendants 2,13..17 on 0,3,5,7,9,11
CELL18_EDGES = [[0, 1], [1, 3], [3, 4], [4, 5], [5, 6], [6, 7], [7, 8], [8, 9], [9, 10], [10, 11], [11, 12],
                [12, 0], [0, 2], [3, 13], [5, 14], [7, 15], [9, 16], [11, 17]]


def motif_pattern(m):
    kind, size = MOTIF_SHAPES[m]
    if kind == "path":
        return W.path(size)
    if kind == "cycle":
        return W.cycle(size)
    if kind == "claw":  # centre 0, leaves 1..3
        return W.star(3)
    if kind == "cell18":
        return W.Pattern(18, CELL18_EDGES, "M18-O-6")
    # 2x3 grid: 0-1-2 over 3-4-5
    return W.Pattern(6, [[0, 1], [1, 2], [3, 4], [4, 5], [0, 3], [1, 4], [2, 5]], "2x3")


def motif_rows(g, m):
    p = motif_pattern(m)
    rows, _ = oracle.enumerate_embeddings(g.n, g.edges, p.n, p.edges)
    return rows


def execute(g, plan):
    adj = set()
    for u, v in g.edges.tolist():
        if u != v:
            adj.add((u, v))
            adj.add((v, u))
    R = [(v,) for v in range(g.n)]
    cache = {}
    for st in plan["steps"]:
        out = []
        if st["motif"] < 0:
            for r in R:
                if all((r[a], r[b]) in adj for a, b in st["edges"]):
                    out.append(r)
            R = out
            continue
        m = st["motif"]
        if m not in cache:
            tab = motif_rows(g, m)
            index = {}
            for row in tab.tolist():
                index.setdefault((st["key_pos"], row[st["key_pos"]]), []).append(row)
            cache[m] = tab
        tab = cache[m]
        index = {}
        kp = st["key_pos"]
        for row in tab.tolist():
            index.setdefault(row[kp], []).append(row)
        c_in = st["c_in"]
        for r in R:
            for mr in index.get(r[st["key_col"]], []):
                if any(mr[pos] != r[col] for col, pos in st["eq"]):
                    continue
                new = [mr[p] for p in st["new_pos"]]
                if any(x in r for x in new):
                    continue
                full = r + tuple(new)
                if all((full[a], full[b]) in adj for a, b in st["edges"]):
                    out.append(full)
        R = out
    k = plan["k"]
    col_of = plan["col_of"]
    rows = np.array([[r[col_of[j]] for j in range(k)] for r in R], dtype=np.int32).reshape(-1, k)
    if len(rows):
        rows = rows[np.lexsort(rows.T[::-1])]
    return rows
