#!/usr/bin/env python3
"""Benchmark: embeddings/s of the full hot path on one MI355X.

Headline workload (the scaling configuration): the heavy-hex lattices
HH(28,28), HH(56,56), HH(90,90) (973, 3906 and 10103 vertices) and the
100x100 square grid, each with the patterns P8, P12, P16, C12, four seeded
16-vertex Pruefer trees (max degree within the lattice's) and the 2x3 / 3x3
grids, every embedding enumerated as a sorted int32 table.  One step = for
each lattice, build the resident data graph (CSR, bitmap, motif tables) and
enumerate every pattern through the plain path (host decomposition, one join
launch per step, the sort tiers), i.e. every row of the hot path.  Pairs whose
intermediate tables pass ~1e8 rows by far (P12, P16 and the trees on the
grid: 1e9..6e10 embeddings) are not in the step; they run once in count+hash
mode (``over_budget``).  Inputs are host arrays of a few KB, copied by the
library inside the step.

Before anything is timed, every pair's count and multiset row hash (GPU,
count+hash mode) is compared with the CPU oracle's stored values
(tests/golden/oracle_counts.json, written by tests/golden/make_golden.py).

Prints one JSON line with, besides the headline:
* ``cases``: per pair, embeddings and the join / sort kernels' time and
  bandwidth (algorithmic bytes) in the fastest step;
* ``roofline``: the dominant kernel of the timed steps (HIP events around
  every launch on the library's stream), algorithmic bytes over launch time;
* ``over_budget``: the grid pairs above, count+hash mode, against the oracle;
* ``batched``: the batched form against one plain launch per pattern on the
  device-scale configuration (HH(7,19), 64 lattice-subgraph patterns);
* ``served``: Poisson traces on HH(56,56) (circuit patterns of 4..60 qubits,
  caps {1, 1000, all}) through the server and one plain solve at a time, at
  100..5000 queries/s, with p50/p99 latency and queries/s;
* ``cpu_baseline``: the CPU oracle on the headline workload in table mode
  (enumerate + sort), on every host thread (root ranges split across
  threads) and on one thread.
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
METRIC = "embeddings/sec + achieved HBM GB/s; batched/served vs plain per-pattern runs"
# counter summaries of the dominant kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by a plain copy's readings); used only while the kernel source is the
# one the counters were taken on
TRAFFIC_PROFILES = {"ejf_kernel": os.path.join(ROOT, "profiles", "ejf_kernel_config3.md"),
                    "sort": os.path.join(ROOT, "profiles", "sort_config3.md")}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (as the roofline counts launches) from
    its committed counter summary, or None when it is missing, gives none, or
    the kernel source has changed since."""
    import hashlib
    try:
        txt = open(TRAFFIC_PROFILES[kernel]).read()
    except (OSError, KeyError):
        return None
    vals = {}
    for line in txt.splitlines():
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2508_21287_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if vals.get("kernels_hip_sha256") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--no-serve", dest="serve", action="store_false", help="skip the served traces")
    ap.add_argument("--no-over-budget", dest="hbm", action="store_false",
                    help="skip the over-budget grid pairs (count+hash mode)")
    ap.add_argument("--serve-queries", type=int, default=300, help="queries per arrival rate in the served traces")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--batched-config4", action="store_true",
                    help="refused: the batched run of 256 circuit patterns on HH(28,28) stays off the GPU")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the headline steps (no comparison legs), for profilers")
    ap.add_argument("--config2", action="store_true",
                    help="instead of the benchmark line, the device-scale case: HH(7,19) x 64 lattice-subgraph "
                         "patterns, batched vs plain")
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
    ap.add_argument("--pattern-size", type=int, default=60, help="motif-set study: heavy-hex pattern vertices")
    ap.add_argument("--grid-pattern-size", type=int, default=16,
                    help="motif-set study: grid pattern vertices (tree-like grid subgraphs explode beyond ~20)")
    ap.add_argument("--patterns", type=int, default=8)
    return ap.parse_args()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_tables(g, pats, threads, lib):
    """The oracle in table mode on every pattern: each pattern's roots split
    into `threads` contiguous ranges run on host threads (the oracle's C code
    releases the interpreter lock), the ranges' sorted tables concatenated in
    root order (= the pattern's sorted table).  Returns the rows produced."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    rows = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for p in pats:
            cuts = np.linspace(0, g.n, threads + 1).astype(int)
            futs = [ex.submit(oracle.enumerate_embeddings, g.n, g.edges, p.n, p.edges, -1, lib,
                              (int(cuts[i]), int(cuts[i + 1]))) for i in range(threads)]
            parts = [f.result()[0] for f in futs]
            rows += sum(len(t) for t in parts)
            del parts
    return rows


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
            # one blocking call per completion, in completion order (the
            # call releases the interpreter lock while it waits)
            while len(done) < n_queries:
                t, r, code = srv.wait_any(-1)
                now = time.perf_counter() - t0
                if code not in (0, budget_code):
                    raise dm.DMError(code, f"served query failed with {code}")
                if code == budget_code:
                    state["rejected"] += 1
                done[t] = now
                if r is not None:
                    state["rows"] += r.rows
                    r.free()

        th = threading.Thread(target=waiter)
        th.start()
        for i in range(n_queries):
            wait_until(t0, arrivals[i])
            p = pats[i]
            tickets.append(srv.submit(p.n, p.edges, int(caps[i])))
        th.join()
        el = time.perf_counter() - t0
        srv.stop()
        lat = np.array([done[tickets[i]] - arrivals[i] for i in range(n_queries)])
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


def served_block(dm, W, ctx, n_queries, rates=(100, 300, 1000, 3000, 5000)):
    """The served configuration: HH(56,56) resident, at each arrival rate an
    open-loop Poisson trace of circuit patterns (4..60 qubits, caps {1, 1000,
    all}) through the server (continuous batching on 2 streams, admission by
    predicted table memory, 8 GiB per query) and, on the same trace, one plain
    solve at a time within the same 8 GiB."""
    import numpy as np
    budget = 8 << 30
    dg = None
    out = []
    for rate in rates:
        g, arrivals, pats, caps = W.config5(float(rate), n_queries=n_queries)
        if dg is None:
            dg = dm.DataGraph(ctx, g.n, g.edges)
            replay(dm, dg, np.arange(8) * 1e-3, pats[:8], caps[:8], budget)  # warm-up
        # both legs find every query's plan in the context's plan cache (the
        # server's leg runs first: cold plans would be charged to it alone)
        for p in pats:
            dg.estimate(p.n, p.edges)
        lat_s, el_s, rej_s, lat_p, el_p, rej_p, rows = replay(dm, dg, arrivals, pats, caps, budget)
        out.append({"rate_per_s": rate, "queries": n_queries, "rows": int(rows),
                    "refused": rej_s, "p50_ms": 1e3 * float(np.percentile(lat_s, 50)),
                    "p99_ms": 1e3 * float(np.percentile(lat_s, 99)), "qps": n_queries / el_s,
                    "plain_refused": rej_p, "plain_p50_ms": 1e3 * float(np.percentile(lat_p, 50)),
                    "plain_p99_ms": 1e3 * float(np.percentile(lat_p, 99)), "plain_qps": n_queries / el_p})
        print(f"bench: served {rate}/s done", file=sys.stderr, flush=True)
    dg.free()
    return {"trace": f"HH(56,56) (3906 vertices), {n_queries} circuit-pattern queries of 4-60 qubits per rate, "
                     "Poisson arrivals, caps {1, 1000, all}, 8 GiB per query, 2 server streams",
            "rates": out,
            "qps_ge_plain_every_rate": all(r["qps"] >= r["plain_qps"] for r in out),
            "p99_le_plain_every_rate": all(r["p99_ms"] <= r["plain_p99_ms"] for r in out)}


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


def timed_steps(torch, step, steps, warmup):
    """W untimed then K timed calls of step(); returns (seconds, [results])."""
    for _ in range(warmup):
        step()
    # the interpreter's cyclic collector walks every live object (torch holds
    # about a million) in its full passes, a 40-70 ms pause every few steps;
    # move the objects alive now out of its reach, as a serving process would
    gc.collect()
    gc.freeze()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def step_accounting(dm, res):
    sm = dm.summarize(res)  # one call for all results' counts and launch accounting
    return (int(sm["total"].sum()), float(sm["join_ms"].sum()), int(sm["join_bytes"].sum()),
            int(sm["join_launches"].sum()), float(sm["sort_ms"].sum()), int(sm["sort_bytes"].sum()),
            int(sm["sort_launches"].sum()))


def roofline_of(acc, steps):
    """The dominant kernel of the timed steps: the persistent join launch or
    the sort (its tiers, one launch set per step), by summed device time."""
    join_ms = sum(a[1] for a in acc)
    join_b = sum(a[2] for a in acc)
    join_l = sum(a[3] for a in acc)
    sort_ms = sum(a[4] for a in acc)
    sort_b = sum(a[5] for a in acc)
    if join_ms >= sort_ms:
        name, ms, byts, launches = "batch_kernel", join_ms, join_b, max(join_l, 1)
        desc = "batch_kernel (persistent expand-join-filter over all patterns)"
    else:
        name, ms, byts, launches = "sort", sort_ms, sort_b, max(steps, 1)
        desc = "sort tiers (per-root-segment LDS sorts, one launch set per step)"
    ach = (byts / 1e9) / (ms / 1e3) if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(name), "kernel": desc, "launches": launches,
            "avg_launch_us": 1e3 * ms / launches, "bytes_per_launch": byts / launches,
            "join_ms_per_step": join_ms / max(steps, 1), "sort_ms_per_step": sort_ms / max(steps, 1)}


def config2_line(dm, W, ctx, torch, args):
    """The device-scale case (HH(7,19), 64 lattice-subgraph patterns of 8..30
    vertices): batched steps (build + batch) and plain steps."""
    g, pats = W.config2()
    specs = [(p.n, p.edges) for p in pats]

    def step(batch=True):
        dg = dm.DataGraph(ctx, g.n, g.edges)
        res = dg.enumerate_batch(specs, profile=True) if batch else \
            [dg.enumerate(n, e, profile=True) for n, e in specs]
        acc = step_accounting(dm, res)
        dm.free_results(res)
        dg.free()
        return acc

    el, acc = timed_steps(torch, step, args.steps, args.warmup)
    emb = sum(a[0] for a in acc)
    tp, accp = timed_steps(torch, lambda: step(False), max(1, min(args.steps, 3)), 1)
    pemb = sum(a[0] for a in accp)
    out = {"config2": "HH(7,19) (163 vertices) x 64 lattice-subgraph patterns of 8-30 vertices",
           "embeddings_per_s": emb / el, "ms_per_step": 1e3 * el / args.steps,
           "plain_embeddings_per_s": pemb / tp, "batched_over_plain": (emb / el) / (pemb / tp),
           "roofline": roofline_of(acc, args.steps)}
    if args.serve:
        out["served"] = serve_trace(dm, ctx, g, pats)
    print(json.dumps(out), flush=True)


GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_counts.json")
LATTICES = ("HH28", "HH56", "HH90", "GRID100")


def over_budget(lattice, p):
    """Pairs far beyond ~1e8 rows: P12 (1.1e9 embeddings), P16 (6e10) and the
    16-vertex trees (1e9..9e9) on the 100x100 grid."""
    return lattice == "GRID100" and (p.name in ("P12", "P16") or p.name.startswith("T16"))


def config3_sets(W):
    """[(lattice, graph, [patterns])] of the scaling configuration."""
    return [(lat,) + W.config3(lat, n_trees=4) for lat in LATTICES]


def golden():
    import json as _j
    return _j.load(open(GOLDEN))["cases"]


def c3_gate(dm, ctx, sets, gold):
    """Every pair (GPU, count+hash mode) against the oracle's stored count and
    multiset hash; returns {key: count} of the headline pairs."""
    counts = {}
    for lat, g, pats in sets:
        dg = dm.DataGraph(ctx, g.n, g.edges)
        for p in pats:
            if over_budget(lat, p):
                continue
            key = f"{lat}/{p.name}"
            want = gold.get(key)
            if want is None:
                raise SystemExit(f"bench.py: no stored oracle value for {key} (run tests/golden/make_golden.py)")
            with dg.enumerate(p.n, p.edges, mode=dm.OUT_COUNT_HASH) as r:
                got = (r.total,) + r.hash()
            if got != (want["count"], int(want["hash_sum"]), int(want["hash_xor"])):
                raise SystemExit(f"bench.py: GPU count/hash of {key} differs from the oracle: {got} vs {want}")
            counts[key] = want["count"]
        dg.free()
    return counts


def c3_step(dm, ctx, sets):
    """One step: per lattice, build the data graph and enumerate every
    headline pattern as a sorted table.  Returns per-pair tuples
    (key, total, join_ms, join_bytes, join_launches, sort_ms, sort_bytes)."""
    acc = []
    for lat, g, pats in sets:
        d = dm.DataGraph(ctx, g.n, g.edges)
        for p in pats:
            if over_budget(lat, p):
                continue
            r = d.enumerate(p.n, p.edges, profile=True)
            acc.append((f"{lat}/{p.name}", r.total) + r.timing())
            r.free()
        d.free()
    return acc


def c3_roofline(acc_steps, steps):
    """The dominant kernel of the timed steps (per-launch join or the sort
    tiers) by summed device time: algorithmic bytes over launch time."""
    jm = sum(a[2] for s in acc_steps for a in s)
    jb = sum(a[3] for s in acc_steps for a in s)
    jl = sum(a[4] for s in acc_steps for a in s)
    sm = sum(a[5] for s in acc_steps for a in s)
    sb = sum(a[6] for s in acc_steps for a in s)
    sl = sum(1 for s in acc_steps for a in s if a[6] > 0)
    if jm >= sm:
        name, ms, byts, launches = "ejf_kernel", jm, jb, max(jl, 1)
        desc = "ejf_kernel (per-launch expand-join-filter, one launch per join step)"
    else:
        name, ms, byts, launches = "sort", sm, sb, max(sl, 1)
        desc = "sort tiers (per-root-segment LDS sorts + merge tier, one launch set per pattern)"
    ach = (byts / 1e9) / (ms / 1e3) if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(name), "kernel": desc, "launches": launches,
            "avg_launch_us": 1e3 * ms / launches, "bytes_per_launch": byts / launches,
            "join_ms_per_step": jm / max(steps, 1), "sort_ms_per_step": sm / max(steps, 1),
            "join_GBps": (jb / 1e9) / (jm / 1e3) if jm else None,
            "sort_GBps": (sb / 1e9) / (sm / 1e3) if sm else None}


def c3_cases(acc_steps):
    """Per pair, the fastest step's join and sort figures."""
    out = {}
    for s in acc_steps:
        for key, tot, jm, jb, jl, sm, sb in s:
            cur = out.get(key)
            t = jm + sm
            if cur is None or t < cur["join_ms"] + (cur["sort_ms"] or 0):
                out[key] = {"embeddings": tot, "join_ms": jm, "join_launches": jl,
                            "join_GBps": (jb / 1e9) / (jm / 1e3) if jm else None,
                            "sort_ms": sm or None, "sort_GBps": (sb / 1e9) / (sm / 1e3) if sm else None}
    return out


def over_budget_block(dm, ctx, sets, gold):
    """The grid pairs beyond the table budget, once each in count+hash mode
    (root ranges chunked to the memory budget), against the oracle."""
    import torch
    out = {}
    for lat, g, pats in sets:
        todo = [p for p in pats if over_budget(lat, p)]
        if not todo:
            continue
        dg = dm.DataGraph(ctx, g.n, g.edges)
        for p in todo:
            key = f"{lat}/{p.name}"
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with dg.enumerate(p.n, p.edges, mode=dm.OUT_COUNT_HASH, profile=True) as r:
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                got = (r.total,) + r.hash()
                st = r.stats()
            want = gold.get(key)
            ok = None if want is None else got == (want["count"], int(want["hash_sum"]), int(want["hash_xor"]))
            out[key] = {"embeddings": got[0], "wall_ms": 1e3 * el, "embeddings_per_s": got[0] / el,
                        "join_ms": st["join_ms"], "join_GBps": (st["join_bytes"] / 1e9) / (st["join_ms"] / 1e3)
                        if st["join_ms"] else None, "chunks": st["chunks"], "matches_oracle": ok}
            print(f"bench: over-budget {key} {got[0]} in {1e3 * el:.0f} ms", file=sys.stderr, flush=True)
            if ok is False:
                raise SystemExit(f"bench.py: GPU count/hash of {key} differs from the oracle")
        dg.free()
    return out


def c3_cpu_baseline(sets, budget_s=12.0):
    """The oracle as it stands (C backtracking + qsort, table mode) on the
    headline pairs: all of them on every host thread (root ranges split),
    and pairs in order on one thread until ~budget_s."""
    import oracle
    lib = oracle.load()
    nt = host_threads()
    pairs = [(g, p) for lat, g, pats in sets for p in pats if not over_budget(lat, p)]
    t0 = time.perf_counter()
    rows_n = sum(oracle_tables(g, [p], nt, lib) for g, p in pairs)
    el_n = time.perf_counter() - t0
    rows_1, used, t1 = 0, 0, time.perf_counter()
    for g, p in pairs:
        rows_1 += oracle_tables(g, [p], 1, lib)
        used += 1
        if time.perf_counter() - t1 > budget_s:
            break
    el_1 = time.perf_counter() - t1
    return {"value": rows_n / el_n, "unit": "embeddings/s", "cores": nt, "kind": "oracle",
            "sample": f"every headline pair ({len(pairs)}), table mode (enumerate + sort), {nt} threads over "
                      f"root ranges: {rows_n} rows in {el_n:.1f} s; 1 thread: the first {used} pairs, {rows_1} "
                      f"rows in {el_1:.1f} s",
            "value_1thread": rows_1 / el_1, "cpu_model": cpu_model()}


def batched_block(dm, W, ctx, torch, steps):
    """Batched form vs one plain launch per pattern, device-scale
    configuration (HH(7,19), 64 lattice-subgraph patterns of 8..30 vertices),
    both including the data-graph build."""
    g, pats = W.config2()
    specs = [(p.n, p.edges) for p in pats]

    def step(batch=True):
        dg = dm.DataGraph(ctx, g.n, g.edges)
        res = dg.enumerate_batch(specs, profile=True) if batch else \
            [dg.enumerate(n, e, profile=True) for n, e in specs]
        acc = step_accounting(dm, res)
        dm.free_results(res)
        dg.free()
        return acc

    el, acc = timed_steps(torch, step, steps, 3)
    emb = sum(a[0] for a in acc)
    tp, accp = timed_steps(torch, lambda: step(False), 3, 1)
    pemb = sum(a[0] for a in accp)
    if emb // steps != pemb // 3:
        raise SystemExit("bench.py: batched and plain runs disagree on the embedding count")
    # the launch-shape autotuner on a resident copy of the data graph (not
    # timed with the steps: the tuned shape stays on that graph)
    dg = dm.DataGraph(ctx, g.n, g.edges)
    best, tried = dg.autotune_batch(specs, reps=3)
    default = [t for t in tried if t["block_threads"] == 256 and t["backoff"] == 15]
    default = min(default, key=lambda t: abs(t["grid"] - 256)) if default else None
    dg.free()
    return {"workload": "HH(7,19) (163 vertices) x 64 lattice-subgraph patterns of 8-30 vertices, "
                        "data-graph build + every pattern per step",
            "batched_embeddings_per_s": emb / el, "batched_ms_per_step": 1e3 * el / steps,
            "plain_embeddings_per_s": pemb / tp, "plain_ms_per_step": 1e3 * tp / 3,
            "batched_over_plain": (emb / el) / (pemb / tp),
            "batch_kernel": roofline_of(acc, steps),
            "autotune": {"best": best, "default_shape_ms": default["ms"] if default else None,
                         "shapes_tried": len(tried), "note": "ms = one batched call on the resident graph, "
                                                            "count+hash mode, median of 3"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.batched_config4:
        raise SystemExit("bench.py: the batched run of 256 circuit patterns on HH(28,28) stays off the GPU: the "
                         "batched call hung once on a subset of it and no cause has been shown")
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
    if args.config2:
        config2_line(dm, W, ctx, torch, args)
        return

    sets = config3_sets(W)
    gold = golden()
    if not args.profile_run:
        counts = c3_gate(dm, ctx, sets, gold)
        expect = sum(counts.values())
        print(f"bench: parity gate passed ({expect} embeddings, {len(counts)} pairs)", file=sys.stderr, flush=True)
    el, acc = timed_steps(torch, lambda: c3_step(dm, ctx, sets), args.steps, args.warmup)
    emb = sum(a[1] for s in acc for a in s)
    if not args.profile_run and emb != expect * args.steps:
        raise SystemExit(f"bench.py: timed steps produced {emb} rows, expected {expect * args.steps}")
    n_pairs = len(acc[0]) if acc else 0
    out = {
        "metric": METRIC,
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
        "config": {"workload": "heavy-hex HH(28,28) / HH(56,56) / HH(90,90) (973 / 3906 / 10103 vertices) and the "
                               "100x100 grid x {P8, P12, P16, C12, 4 seeded 16-vertex Pruefer trees, 2x3 and 3x3 "
                               f"grids}} ({n_pairs} pairs; P12, P16 and the trees on the grid are in over_budget), "
                               "full enumeration, sorted int32 tables",
                   "mode": "plain", "embeddings_per_step": emb // max(args.steps, 1),
                   "step": "per lattice: data-graph build + motif tables, then per pattern: plan + join launches "
                           "+ sort"},
        "roofline": c3_roofline(acc, args.steps),
    }
    if args.profile_run:
        print(json.dumps(out), flush=True)
        return
    out["cases"] = c3_cases(acc)
    print("bench: headline steps done", file=sys.stderr, flush=True)
    if args.hbm:
        out["over_budget"] = over_budget_block(dm, ctx, sets, gold)
    out["batched"] = batched_block(dm, W, ctx, torch, 20)
    print("bench: batched vs plain done", file=sys.stderr, flush=True)
    if args.serve:
        out["served"] = served_block(dm, W, ctx, args.serve_queries)
    if not args.no_cpu:
        out["cpu_baseline"] = c3_cpu_baseline(sets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
