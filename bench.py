#!/usr/bin/env python3
"""Benchmark: embeddings/s of the full hot path on one MI355X.

Workload: the device-scale configuration -- heavy-hex lattice HH(7,19)
(163 vertices, 186 edges) and 64 seeded connected lattice-subgraph patterns
of 8..30 vertices (random BFS + thinning), full enumeration as sorted int32
tables.  One step = build the resident data graph (CSR, bitmap, motif tables
M3/M4/M12-O) + decompose and enumerate all 64 patterns + canonical sort, i.e.
every row of the hot path.  Inputs are host arrays of a few KB, copied by the
library at the start of the step.

Prints one JSON line.  The roofline entry is for the dominant kernel (the
expand-join-filter launches): algorithmic bytes (each table read once and
written once) over the summed launch durations measured with HIP events on
the library's stream during the timed steps.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# counter summary of the dominant kernel on this workload (rocprofv3 FETCH_SIZE /
# WRITE_SIZE, scaled by a plain copy's readings); used only while the kernel
# source is the one the counters were taken on
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "batch_kernel_hh7x19_64pat.md")


def measured_traffic():
    """HBM bytes per dispatch of the dominant kernel from the committed counter
    summary, or None when it is missing or the kernel source has changed."""
    import hashlib
    try:
        txt = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2508_21287_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if vals.get("kernels_hip_sha256") != sha or "traffic_bytes_per_dispatch" not in vals:
        return None
    return float(vals["traffic_bytes_per_dispatch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--mode", choices=["batch", "plain"], default="batch")
    ap.add_argument("--no-serve", dest="serve", action="store_false",
                    help="skip the served-trace measurement")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the benchmark line, print one JSON line per large-table case "
                         "(10k-vertex lattices) with the join and sort kernels' bandwidth")
    ap.add_argument("--motif-sets", action="store_true",
                    help="instead of the benchmark line, time random lattice-subgraph patterns under each "
                         "motif set (with and without building the motif tables) and count the join "
                         "iterations, one JSON line per (topology, motif set)")
    ap.add_argument("--served-sweep", action="store_true",
                    help="instead of the benchmark line, replay Poisson traces of circuit patterns on HH(56,56) "
                         "at 100..5000 queries/s through the server and one at a time, one JSON line per rate")
    ap.add_argument("--queries", type=int, default=500, help="served sweep: queries per rate")
    ap.add_argument("--batched-config4", action="store_true",
                    help="instead of the benchmark line, time 256 circuit patterns on HH(28,28) as one "
                         "batched call vs 256 plain calls")
    ap.add_argument("--pattern-size", type=int, default=60, help="motif-set study: heavy-hex pattern vertices")
    ap.add_argument("--grid-pattern-size", type=int, default=16,
                    help="motif-set study: grid pattern vertices (tree-like grid subgraphs explode beyond ~20)")
    ap.add_argument("--patterns", type=int, default=8)
    return ap.parse_args()


def cpu_baseline(g, pats, budget_s=10.0):
    """The oracle as it stands (single-threaded C backtracking) on the same
    workload, repeated until ~budget_s of CPU time (bounded sample)."""
    import oracle
    oracle.load()
    total = 0
    reps = 0
    t0 = time.perf_counter()
    while True:
        for p in pats:
            c, _, _ = oracle.count_hash(g.n, g.edges, p.n, p.edges)
            total += c
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 200:
            break
    return {"value": total / el, "unit": "embeddings/s", "cores": 1, "kind": "oracle",
            "sample": f"all 64 patterns x {reps} repetitions ({el:.1f} s), count+hash mode, 1 thread"}


def wait_until(t0, t):
    """Wait until perf_counter() - t0 reaches t: sleep (which lets the other
    Python threads run) and spin only the last 100 us."""
    while True:
        dt = t - (time.perf_counter() - t0)
        if dt <= 0:
            return
        if dt > 2e-4:
            time.sleep(dt - 1e-4)


def replay(dm, dg, arrivals, pats, caps, mem_budget=0):
    """Open-loop replay of one trace: through the server (continuous batching,
    2 streams) and, on the same queries, one plain solve at a time (FIFO, no
    overlap).  Latency = completion - arrival, also for a query the library
    refuses (over its memory budget: counted as rejected).  Returns
    ``(server_latencies, server_seconds, server_rejected, plain_latencies,
    plain_seconds, plain_rejected, rows)``; rows = rows delivered by the
    server."""
    import threading
    import numpy as np
    n_queries = len(pats)
    budget_code = -6  # DM_ERR_BUDGET_EXCEEDED

    def run_server():
        srv = dm.Server(dg, n_streams=2, max_batch=64, mem_budget=mem_budget)
        done = {}
        tickets = []
        state = {"rejected": 0, "rows": 0}
        t0 = time.perf_counter()

        def waiter():
            # poll every outstanding ticket (timeout 0) so completions are
            # seen in whatever order they happen
            pending = set()
            seen = 0
            while len(done) < n_queries:
                while seen < len(tickets):
                    pending.add(seen)
                    seen += 1
                for i in list(pending):
                    try:
                        r = srv.wait(tickets[i], 0)
                    except dm.DMError as e:
                        if e.code == -10:  # not finished yet
                            continue
                        if e.code != budget_code:
                            raise
                        state["rejected"] += 1
                        r = None
                    done[i] = time.perf_counter() - t0
                    if r is not None:
                        state["rows"] += r.rows
                        r.free()
                    pending.discard(i)
                time.sleep(0.0001)

        th = threading.Thread(target=waiter)
        th.start()
        for i in range(n_queries):
            wait_until(t0, arrivals[i])
            p = pats[i]
            tickets.append(srv.submit(p.n, p.edges, int(caps[i])))
        th.join()
        el = time.perf_counter() - t0
        srv.stop()
        lat = np.array([done[i] - arrivals[i] for i in range(n_queries)])
        return lat, el, state["rejected"], state["rows"]

    def run_plain():
        # the server runs each query within its budget: so do the plain solves
        opts = {"mem_budget": mem_budget, "result_mb": mem_budget >> 20} if mem_budget else {}
        t0 = time.perf_counter()
        fin = []
        rejected = 0
        for i in range(n_queries):
            wait_until(t0, arrivals[i])
            p = pats[i]
            try:
                dg.enumerate(p.n, p.edges, int(caps[i]), **opts).free()
            except dm.DMError as e:
                if e.code != budget_code:
                    raise
                rejected += 1
            fin.append(time.perf_counter() - t0)
        el = time.perf_counter() - t0
        return np.array(fin) - arrivals, el, rejected

    lat_s, el_s, rej_s, rows = run_server()
    lat_p, el_p, rej_p = run_plain()
    return lat_s, el_s, rej_s, lat_p, el_p, rej_p, rows


def serve_trace(dm, ctx, g, pats, rate=4000.0, n_queries=512, seed=4000):
    """Poisson trace of the benchmark patterns (caps drawn from {1, 1000,
    all}) through the server vs the same trace solved one query at a time."""
    import numpy as np
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_queries))
    order = rng.integers(0, len(pats), size=n_queries)
    caps = rng.choice(np.array([1, 1000, -1]), size=n_queries)
    dg = dm.DataGraph(ctx, g.n, g.edges)
    qp = [pats[i] for i in order]
    replay(dm, dg, arrivals, qp, caps)  # warm-up
    lat_s, el_s, _, lat_p, el_p, _, _ = replay(dm, dg, arrivals, qp, caps)
    dg.free()
    return {"trace": f"{n_queries} queries, Poisson {rate:.0f}/s, caps {{1,1000,all}}, same 64 patterns",
            "p50_ms": 1e3 * float(np.percentile(lat_s, 50)), "p99_ms": 1e3 * float(np.percentile(lat_s, 99)),
            "qps": n_queries / el_s,
            "plain_p50_ms": 1e3 * float(np.percentile(lat_p, 50)),
            "plain_p99_ms": 1e3 * float(np.percentile(lat_p, 99)), "plain_qps": n_queries / el_p}


def batched_config4(dm, W, ctx, reps=5):
    """256 circuit patterns (4-40 qubits) on HH(28,28): one batched call (the
    persistent join launch for all patterns, then the sort tiers) vs 256
    plain calls on the same stream; full tables.  One JSON line."""
    import numpy as np
    import torch
    g, pats = W.config4(256)
    specs = [(p.n, p.edges) for p in pats]
    dg = dm.DataGraph(ctx, g.n, g.edges)
    rows = 0
    for _ in range(2):
        res = dg.enumerate_batch(specs)
        rows = sum(r.rows for r in res)
        for r in res:
            r.free()
    tb, tp = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in dg.enumerate_batch(specs):
            r.free()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        for p in pats:
            dg.enumerate(p.n, p.edges).free()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    b, q = float(np.median(tb)), float(np.median(tp))
    print(json.dumps({"batched": "HH(28,28) x 256 circuit patterns 4-40 qubits", "rows": int(rows),
                      "batch_ms": 1e3 * b, "plain_ms": 1e3 * q, "batch_embeddings_per_s": rows / b,
                      "plain_embeddings_per_s": rows / q, "batched_over_plain": q / b}), flush=True)
    dg.free()


def served_sweep(dm, W, ctx, n_queries):
    """Served workload on HH(56,56): at each arrival rate, an open-loop trace of
    circuit patterns (4-60 qubits, caps {1, 1000, all}) through the server vs
    plain solves; each query runs within the server's default 8 GiB budget
    (a result beyond it is refused).  One JSON line per rate."""
    import numpy as np
    budget = 8 << 30
    dg = None
    for rate in (100, 300, 1000, 3000, 5000):
        g, arrivals, pats, caps = W.config5(float(rate), n_queries=n_queries)
        if dg is None:
            dg = dm.DataGraph(ctx, g.n, g.edges)
            w_arr = np.arange(8) * 1e-3
            replay(dm, dg, w_arr, pats[:8], caps[:8], budget)  # warm-up
        lat_s, el_s, rej_s, lat_p, el_p, rej_p, rows = replay(dm, dg, arrivals, pats, caps, budget)
        print(json.dumps({"served": "HH(56,56) circuit patterns 4-60 qubits", "rate_per_s": rate,
                          "queries": n_queries, "rows": int(rows), "rejected_over_budget": rej_s,
                          "p50_ms": 1e3 * float(np.percentile(lat_s, 50)),
                          "p99_ms": 1e3 * float(np.percentile(lat_s, 99)), "qps": n_queries / el_s,
                          "plain_p50_ms": 1e3 * float(np.percentile(lat_p, 50)),
                          "plain_p99_ms": 1e3 * float(np.percentile(lat_p, 99)), "plain_qps": n_queries / el_p,
                          "plain_rejected_over_budget": rej_p}), flush=True)
    dg.free()


def sweep(dm, W, ctx, reps=3):
    """HBM regime: large join/sort tables on the 10k-vertex lattices."""
    import torch
    cases = [("GRID100", W.path(8), dm.OUT_TABLE), ("GRID100", W.cycle(12), dm.OUT_COUNT_HASH),
             ("GRID100", W.path(10), dm.OUT_COUNT_HASH), ("HH90", W.path(16), dm.OUT_TABLE),
             ("HH90", W.prufer_tree(16, 2), dm.OUT_TABLE)]
    lat = W.config3_lattices()
    built = {}
    for lname, p, mode in cases:
        if lname not in built:
            g = lat[lname]
            built[lname] = (g, dm.DataGraph(ctx, g.n, g.edges))
        g, dg = built[lname]
        dg.enumerate(p.n, p.edges, mode=mode).free()  # warm-up, sizes the workspace
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            r = dg.enumerate(p.n, p.edges, mode=mode, profile=True)
            el = time.perf_counter() - t0
            st = r.stats()
            tot = r.total
            r.free()
            if best is None or el < best[0]:
                best = (el, st, tot)
        el, st, tot = best
        jg = st["join_bytes"] / 1e9 / (st["join_ms"] / 1e3) if st["join_ms"] else 0.0
        sg = st["sort_bytes"] / 1e9 / (st["sort_ms"] / 1e3) if st["sort_ms"] else 0.0
        print(json.dumps({"sweep": f"{lname} {p.name}", "mode": "table" if mode == dm.OUT_TABLE else "count+hash",
                          "embeddings": tot, "wall_ms": 1e3 * el, "embeddings_per_s": tot / el,
                          "join_ms": st["join_ms"], "join_launches": st["join_launches"],
                          "join_bytes": st["join_bytes"], "join_GBps": jg, "join_frac_hbm": jg / HBM_PEAK_GBS,
                          "sort_ms": st["sort_ms"], "sort_bytes": st["sort_bytes"], "sort_GBps": sg,
                          "step_rows": st["step_rows"], "retries": st["retries"], "chunks": st["chunks"]}),
              flush=True)
    for _, dg in built.values():
        dg.free()


def motif_sets(dm, W, ctx, k_hh, k_grid, n_patterns):
    """Runtime and join iterations per motif set (the motif-selection study):
    random connected subgraphs (random BFS + thinning, seeds 1000..) of the
    4485-vertex heavy-hex lattice (k_hh vertices) and the 3600-vertex grid
    (k_grid vertices), count+hash mode.  'total' includes building the motif tables of the set
    (a fresh data graph per set), 'query' excludes it."""
    import numpy as np
    import torch
    sets = {
        "HH(60,60)": [("M2", dm.MOTIF_M2_ONLY), ("M2+M3", dm.MOTIF_M3), ("M2+M4", dm.MOTIF_M4),
                      ("M2+M4-1", dm.MOTIF_M4_1), ("M2+M6", dm.MOTIF_M6), ("M2+M12-O", dm.MOTIF_C12),
                      ("auto", dm.MOTIF_AUTO)],
        "GRID(60,60)": [("M2", dm.MOTIF_M2_ONLY), ("M2+M4", dm.MOTIF_M4), ("M2+M4-O", dm.MOTIF_C4),
                        ("M2+M4-1", dm.MOTIF_M4_1), ("M2+M6-2O", dm.MOTIF_M6_2O | dm.MOTIF_C4),
                        ("auto", dm.MOTIF_AUTO)],
    }
    for gname, g, k in [("HH(60,60)", W.heavy_hex(60, 60), k_hh), ("GRID(60,60)", W.grid(60, 60), k_grid)]:
        adj = W.adjacency_lists(g)
        pats = [W.lattice_subgraph_pattern(g, k, np.random.default_rng(1000 + s), adj=adj)
                for s in range(n_patterns)]
        for sname, mask in sets[gname]:
            tot, qry, its, counts = [], [], [], []
            for p in pats:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                dg = dm.DataGraph(ctx, g.n, g.edges, mask)
                t1 = time.perf_counter()
                try:
                    with dg.enumerate(p.n, p.edges, mode=dm.OUT_COUNT_HASH,
                                      motif_mask=mask if mask != dm.MOTIF_AUTO else 0) as r:
                        st = r.stats()
                        counts.append(r.total)
                        its.append(st["n_steps"])
                    t2 = time.perf_counter()
                    tot.append(1e3 * (t2 - t0))
                    qry.append(1e3 * (t2 - t1))
                except dm.DMError as e:
                    counts.append(None)
                    its.append(None)
                    print(json.dumps({"motif_set": sname, "graph": gname, "pattern": p.name, "error": str(e)}),
                          flush=True)
                dg.free()
            ok = [i for i, c in enumerate(counts) if c is not None]

            def mmm(xs):
                xs = [xs[i] for i in ok]
                return {"mean": float(np.mean(xs)), "min": float(np.min(xs)), "max": float(np.max(xs))} if xs else None
            print(json.dumps({"motif_sets": gname, "set": sname, "pattern_vertices": k, "patterns": len(pats),
                              "completed": len(ok), "total_ms": mmm(tot), "query_ms": mmm(qry),
                              "iterations": mmm(its), "embeddings": mmm(counts)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibrate:
        n = args.copy_calibrate << 18  # int32 elements
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)
        return
    import paper_2508_21287_amd as dm
    from paper_2508_21287_amd import workloads as W

    g, pats = W.config2()
    specs = [(p.n, p.edges) for p in pats]
    ctx = dm.Context(0)
    if args.sweep:
        sweep(dm, W, ctx)
        return
    if args.motif_sets:
        motif_sets(dm, W, ctx, args.pattern_size, args.grid_pattern_size, args.patterns)
        return
    if args.served_sweep:
        served_sweep(dm, W, ctx, args.queries)
        return
    if args.batched_config4:
        batched_config4(dm, W, ctx)
        return

    def step(profile: bool):
        dg = dm.DataGraph(ctx, g.n, g.edges)
        if args.mode == "batch":
            res = dg.enumerate_batch(specs, profile=profile)
        else:
            res = [dg.enumerate(n, e, profile=profile) for n, e in specs]
        sm = dm.summarize(res)  # one call for all results' counts and launch accounting
        tot = int(sm["total"].sum())
        st = [(float(sm["join_ms"].sum()), int(sm["join_bytes"].sum()), int(sm["join_launches"].sum()),
               float(sm["sort_ms"].sum()), int(sm["sort_bytes"].sum()))]
        dm.free_results(res)
        dg.free()
        return tot, st

    for _ in range(args.warmup):
        step(True)
    # the interpreter's cyclic collector walks every live object (torch holds
    # about a million) in its full passes, a 40-70 ms pause every few steps;
    # move the objects alive now out of its reach, as a serving process would
    gc.collect()
    gc.freeze()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    emb = 0
    join_ms = join_bytes = join_launches = sort_ms = sort_bytes = 0
    for _ in range(args.steps):
        tot, st = step(True)
        emb += tot
        for jm, jb, jl, sm, sb in st:
            join_ms += jm
            join_bytes += jb
            join_launches += jl
            sort_ms += sm
            sort_bytes += sb
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    # the same steps with one plain launch sequence per pattern, for comparison
    plain_steps = max(1, min(args.steps, 3))
    saved = args.mode
    args.mode = "plain"
    torch.cuda.synchronize()
    tp = time.perf_counter()
    pemb = 0
    for _ in range(plain_steps):
        pemb += step(False)[0]
    torch.cuda.synchronize()
    tp = time.perf_counter() - tp
    args.mode = saved

    # query-only throughput (data graph resident: the paper's GPU* measure)
    dg = dm.DataGraph(ctx, g.n, g.edges)
    torch.cuda.synchronize()
    tq = time.perf_counter()
    qemb = 0
    for _ in range(args.steps):
        res = dg.enumerate_batch(specs)
        qemb += int(dm.summarize(res)["total"].sum())
        dm.free_results(res)
    torch.cuda.synchronize()
    tq = time.perf_counter() - tq
    dg.free()

    served = serve_trace(dm, ctx, g, pats) if args.serve else None

    ach = (join_bytes / 1e9) / (join_ms / 1e3) if join_ms > 0 else 0.0
    out = {
        "metric": "embeddings/sec + achieved HBM GB/s; batched/served vs plain per-pattern runs",
        "value": emb / el,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "HH(7,19) heavy-hex (163 vertices) x 64 seeded lattice-subgraph patterns "
                               "(8-30 vertices), full enumeration, sorted int32 tables",
                   "mode": args.mode, "embeddings_per_step": emb // max(args.steps, 1),
                   "step": "data-graph build + motif tables + plan + joins + sort"},
        "query_only_embeddings_per_s": qemb / tq,
        "plain_embeddings_per_s": pemb / tp,
        "batched_over_plain": (emb / el) / (pemb / tp) if pemb else None,
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.mode == "batch" else None,
                     "kernel": ("batch_kernel (persistent expand-join-filter over all patterns)"
                                if args.mode == "batch" else "ejf_kernel (expand-join-filter)"),
                     "launches": join_launches, "avg_launch_us": 1e3 * join_ms / max(join_launches, 1),
                     "bytes_per_launch": join_bytes / max(join_launches, 1)},
        "sort": {"ms_total": sort_ms, "bytes": sort_bytes},
    }
    if served is not None:
        out["served"] = served
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, pats)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
