"""Write oracle_counts.json: count + multiset hash of every scaling-config
pair (P8, P12, P16, C12, 16-vertex Pruefer trees, the 2x3 and 3x3 grids on
HH(28,28), HH(56,56), HH(90,90) and GRID(100,100)).  Calls only the CPU
oracle (oracle/), in count+hash mode, with the roots split over host threads,
on the seeded generators.

    python tests/golden/make_golden.py [--threads N] [--missing] [--only GRID100/P16 ...]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_21287_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_counts.json")
LATTICES = ["HH28", "HH56", "HH90", "GRID100"]


def cases():
    """(key, graph, pattern) for every pair; P9 on the grid is kept as an
    extra case below the 10-vertex paths."""
    out = []
    for lat in LATTICES:
        g, pats = W.config3(lat, n_trees=4)
        if lat == "GRID100":
            pats = pats + [W.path(9)]
        for p in pats:
            out.append((f"{lat}/{p.name}", g, p))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--missing", action="store_true", help="only pairs without a stored value")
    args = ap.parse_args()
    old = {}
    if os.path.exists(OUT):
        old = json.load(open(OUT)).get("cases", {})
    todo = cases()
    keys = {key for key, _, _ in todo}
    res = {k: v for k, v in old.items() if k in keys}  # drop pairs no longer in the configuration
    for key, g, p in todo:
        if args.only is not None and key not in args.only:
            continue
        if args.missing and key in res:
            continue
        t = time.time()
        c, hs, hx = oracle.count_hash_threads(g.n, g.edges, p.n, p.edges, args.threads)
        res[key] = {"count": c, "hash_sum": str(hs), "hash_xor": str(hx)}
        print(f"{key}: {c} ({time.time() - t:.1f} s)", flush=True)
        with open(OUT, "w") as f:
            json.dump({"source": "tests/golden/make_golden.py (CPU oracle, count+hash mode)",
                       "cases": dict(sorted(res.items()))}, f, indent=1)


if __name__ == "__main__":
    main()
