"""Benchmark: sampled-source GTEPS of Brandes' forward + backward pass.

Workload (default): Barabasi-Albert graph, n = 2^20, 5 edges per new vertex
(m_u = 5,242,865 undirected edges, int64 row offsets), 4096 sources drawn on
the device from Philox4x64-10 (seed 7, stream 0). One step = draw the 4096
sources + the full forward/backward pass of all of them + the per-vertex sum
of their dependencies (bc_dependencies, BC_OUT_SUM). Inputs (graph) are
resident in HBM before the timed region.

GTEPS = sum over the step's sources of the undirected edges in the source's
component, divided by the step time (Graph500 convention, fwd+bwd counted once).

Printed on one JSON line, beside the headline value:
  per_source  the same pass in the one-source-per-launch form on a subset
  pair_leg    adaptive pair sampling (eps = 0.05, 32 top-degree targets)
  roofline    the dominant kernel against the 8 TB/s HBM peak
  cpu_baseline the CPU oracle on a bounded sample of the same sources
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_1608_04472_amd/csrc/kernels.hpp", "paper_1608_04472_amd/csrc/bcmi.hip"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/hbm_traffic.md), or None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        line = line.strip()
        if not line.startswith("{"):
            continue
        rec = json.loads(line)
        if rec.get("kernel") == kernel and rec.get("workload") == workload and \
                rec.get("source_hash") == kernel_source_hash():
            return rec["hbm_bytes_per_launch"]
    return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def oracle_rate(O, g, sources, comp_edges, seconds, threads):
    """The oracle on `sources`, one source per call, from `threads` threads that
    share the sources out in order (the oracle keeps no global state, and its
    calls release the interpreter lock) until `seconds` have passed; returns
    (sources done, undirected edges of their components, wall seconds)."""
    import threading
    lock = threading.Lock()
    state = {"next": 0, "edges": 0.0}
    t0 = time.perf_counter()

    def work():
        while True:
            with lock:
                i = state["next"]
                if i >= len(sources) or (time.perf_counter() - t0 >= seconds and i >= 2):
                    return
                state["next"] = i + 1
            O.dependencies(g, sources[i:i + 1], full=False, total=True)
            with lock:
                state["edges"] += float(comp_edges[sources[i]])

    pool = [threading.Thread(target=work) for _ in range(threads)]
    for th in pool:
        th.start()
    for th in pool:
        th.join()
    return state["next"], state["edges"], time.perf_counter() - t0


def component_edges(g):
    """Undirected edge count of each vertex's connected component."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row), shape=(g.n, g.n))
    _, lab = connected_components(a, directed=False)
    deg = np.diff(g.row)
    per_comp = np.bincount(lab, weights=deg) / 2
    return per_comp[lab]


def serving_leg(args, bc, gg):
    """200 resident R-MAT graphs (scales 10-18, edge factors 8-32), a Poisson
    stream of queries (graph uniform, target degree-weighted, half source
    queries with c in {2, 5, 10}, half pair queries with eps in {0.05, 0.1}),
    served with continuous batching; latency = result time - arrival time."""
    import numpy as np
    t = time.time()
    graphs = gg.serving_graphs(args.serve_graphs)
    qs = gg.serving_queries(graphs, args.serve_queries, args.serve_rate)
    for q in qs:
        q["k_max"] = args.serve_kmax_pair if q["kind"] == 1 else args.serve_kmax_source
    log("serving: %d graphs (%d CSR entries) and %d queries generated in %.1fs" % (
        len(graphs), sum(g.nnz for g in graphs), len(qs), time.time() - t))
    S = bc.Server(args.serve_budget_gib << 30, args.serve_batch)
    for g in graphs:
        S.add_graph(g.row, g.col)
    N = len(qs)
    results = {}
    i = 0
    t0 = S.now()
    last_log = time.time()
    while len(results) < N:
        now = S.now() - t0
        while i < N and qs[i]["arrival"] <= now:
            q = qs[i]
            S.submit(q["graph"], q["target"], q["kind"], q["seed"], q["k_max"], c=q["c"],
                     eps=q["eps"], rule=bc.BC_PAIR_EPS, arrival_s=t0 + q["arrival"])
            i += 1
        S.step()
        for r in S.poll():
            results[r["id"]] = r
        st = S.stats()
        if st["queued"] + st["active"] == 0 and i < N:
            time.sleep(max(0.0, min(0.002, qs[i]["arrival"] - (S.now() - t0))))
        if time.time() - last_log > 10:
            last_log = time.time()
            log("serving: %d/%d done, %d queued, %d active, %.1fs" % (
                len(results), N, st["queued"], st["active"], S.now() - t0))
    st = S.stats()
    res = [results[k] for k in sorted(results)]
    lat = np.array([(r["done_s"] - r["arrival_s"]) * 1e3 for r in res])
    makespan = max(r["done_s"] for r in res) - t0
    edges = sum(r["samples"] * graphs[q["graph"]].m_undirected for r, q in zip(res, qs))
    out = {
        "workload": "%d R-MAT graphs (scale 10-18, edge factor 8-32, seeds 100-%d), %d queries "
                    "at %.0f q/s Poisson (seed 3), half source (c 2/5/10), half pair "
                    "(eps 0.05/0.1)" % (len(graphs), 99 + len(graphs), N, args.serve_rate),
        "queries": N, "arrival_rate_qps": args.serve_rate,
        "achieved_qps": N / makespan, "makespan_s": makespan,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()), "rounds": st["rounds"],
        "samples_executed": st["samples_executed"], "samples_used": st["samples_used"],
        "batch_fill": st["samples_executed"] / max(1, args.serve_batch * st["rounds"]),
        "capped": int(sum(r["status"] == bc.BC_CAPPED for r in res)),
        "used_sample_gteps_full_search_equiv": edges / makespan / 1e9,
        "resident_bytes": st["resident_bytes"], "workspace_bytes": st["workspace_bytes"],
    }
    if args.serve_dump:
        with open(args.serve_dump, "w") as f:
            for r, q in zip(res, qs):
                g = graphs[q["graph"]]
                f.write(json.dumps(dict(q, n=g.n, m=g.m_undirected, samples=r["samples"],
                                        status=r["status"],
                                        latency_ms=(r["done_s"] - r["arrival_s"]) * 1e3)) + "\n")
    S.close()
    log("serving: p50 %.1f ms, p99 %.1f ms, %.1f q/s achieved over %.1f s, %d rounds" % (
        out["p50_ms"], out["p99_ms"], out["achieved_qps"], makespan, st["rounds"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--graph", default="ba1m")
    ap.add_argument("--sources", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--schedule", default="auto", choices=["auto", "wave", "pair"])
    ap.add_argument("--bottom-up", type=float, default=0.0)
    ap.add_argument("--level-loop", type=int, default=0,
                    help="pair engine: 1 persistent level loops, -1 one launch per level "
                         "phase, 0 auto")
    ap.add_argument("--per-source", type=int, default=16, help="sources for the per-source leg")
    ap.add_argument("--pair-targets", type=int, default=32)
    ap.add_argument("--pair-eps", type=float, default=0.05)
    ap.add_argument("--no-pair", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="threads for the all-cores oracle run (capped by the CPUs this "
                         "process may use)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-graphs", type=int, default=200)
    ap.add_argument("--serve-queries", type=int, default=200,
                    help="prefix of the 20,000-query stream to serve (the whole stream "
                         "exceeds one GPU's capacity)")
    ap.add_argument("--serve-rate", type=float, default=500.0)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--serve-batch", type=int, default=4096,
                    help="samples per server round (power of two, 64..4096)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-dump", default="", help="write per-query results (JSON lines)")
    ap.add_argument("--serve-kmax-source", type=int, default=1024)
    ap.add_argument("--serve-kmax-pair", type=int, default=4096)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy a 1 GiB device buffer once before timing (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1608_04472_amd as bc

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    g = gg.config_graph(args.graph)
    log("graph %s n=%d nnz=%d built in %.1fs" % (args.graph, g.n, g.nnz, time.time() - t0))
    comp_edges = component_edges(g)
    G = bc.Graph(g.row, g.col)
    sched = {"auto": bc.BC_SCHED_AUTO, "wave": bc.BC_SCHED_BATCHED,
             "pair": bc.BC_SCHED_THREADED}[args.schedule]
    G.configure(sched, args.batch, args.bottom_up, 0, args.level_loop)

    K = args.sources
    srcs = torch.empty(K, dtype=torch.int32, device=dev)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    host_src = gg.philox_sources(args.seed, K, g.n)
    edges_per_step = float(comp_edges[host_src].sum())

    def step():
        bc.bc_draw_sources(G, args.seed, 0, K, srcs)
        bc.bc_dependencies(G, srcs, bc.BC_OUT_SUM, out)

    if args.calibrate_copy:
        # a plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # readings give the scale between those counters and bytes moved
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read + 1 GiB written")
    for i in range(args.warmup):
        t = time.time()
        step()
        torch.cuda.synchronize()
        log("warmup %d: %.1f ms" % (i, 1e3 * (time.time() - t)))
    st = G.stats()
    G.profile(True)      # HIP events around every hot launch on the library's stream
    torch.cuda.synchronize()
    t = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    kern = G.profile_read()
    G.profile(False)
    ms = 1e3 * elapsed / args.steps
    gteps = edges_per_step / (elapsed / args.steps) / 1e9
    st = G.stats()
    log("timed %d steps: %.2f ms/step, %.2f GTEPS, schedule %d, batch %d, levels %d" % (
        args.steps, ms, gteps, st["schedule"], st["batch_width"], st["levels"]))
    for k in kern:
        if k["launches"]:
            log("  %-18s %4d launches %9.2f ms  avg %8.1f us  %7.1f GB/s algorithmic" % (
                k["name"], k["launches"], k["ms"], 1e3 * k["ms"] / k["launches"],
                k["algo_bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0))
    dom = max(kern, key=lambda k: k["ms"])
    achieved = dom["algo_bytes"] / (dom["ms"] * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"], "%s-%d-b%d" % (args.graph, K, st["batch_width"]))
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom["name"],
                "avg_launch_us": 1e3 * dom["ms"] / dom["launches"],
                "algo_bytes_per_launch": dom["algo_bytes"] / dom["launches"]}
    sig = next(k for k in kern if k["name"] == "sigma_pull")
    csr_bytes = 8 * (g.n + 1) + 4 * g.nnz
    batches = -(-K // st["batch_width"])
    reach = sig["units_a"] + K * args.steps          # level-0 pairs are the sources
    step_bytes = (2 * csr_bytes * batches * args.steps + 32 * reach + 16 * sig["units_b"]) \
        / args.steps
    step_model = {"algo_bytes": step_bytes, "GBs": step_bytes / (ms * 1e-3) / 1e9,
                  "frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "reached_pairs": reach / args.steps,
                  "dag_edge_pairs": sig["units_b"] / args.steps}
    log("dominant %s: %.1f GB/s (%.1f%% of HBM); whole step %.1f GB/s (%.1f%%)" % (
        dom["name"], achieved, 100 * achieved / HBM_PEAK_GBS, step_model["GBs"],
        100 * step_model["frac"]))

    # ---------------------------------------------------- per-source form
    per_source = None
    if args.per_source > 0:
        P = bc.Graph(g.row, g.col)
        P.configure(bc.BC_SCHED_PER_SOURCE, 0, 0.0)
        ps = srcs[:args.per_source].clone()
        pout = torch.empty(g.n, dtype=torch.float64, device=dev)
        bc.bc_dependencies(P, ps[:2].contiguous(), bc.BC_OUT_SUM, pout)   # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        bc.bc_dependencies(P, ps, bc.BC_OUT_SUM, pout)
        torch.cuda.synchronize()
        pt = time.perf_counter() - t
        pe = float(comp_edges[host_src[:args.per_source]].sum())
        per_source = {"sources": args.per_source, "ms_per_source": 1e3 * pt / args.per_source,
                      "gteps": pe / pt / 1e9,
                      "batched_speedup": gteps / (pe / pt / 1e9)}
        P.close()
        log("per-source: %.2f ms/source, %.3f GTEPS, batched speedup %.1fx" % (
            per_source["ms_per_source"], per_source["gteps"], per_source["batched_speedup"]))

    # ----------------------------------------------------------- pair leg
    pair = None
    if not args.no_pair and args.pair_targets > 0:
        targets = torch.from_numpy(gg.top_degree(g, args.pair_targets)).to(dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        est, k, S, stt = bc.adaptive_pair(G, targets, bc.BC_PAIR_EPS, args.pair_eps, 1.0,
                                          args.seed, 1 << 20)
        torch.cuda.synchronize()
        pt = time.perf_counter() - t
        pst = G.stats()
        kk = k.cpu().numpy()
        pair = {"targets": args.pair_targets, "eps": args.pair_eps, "ms": 1e3 * pt,
                "samples_executed": int(pst["samples_executed"]),
                "samples_used_max": int(kk.max()), "samples_used_min": int(kk.min()),
                "pairs_per_s": pst["samples_executed"] / pt,
                "capped": int((stt.cpu().numpy() == bc.BC_CAPPED).sum())}
        log("pair leg: %.1f ms, %d pairs executed (%.0f pairs/s)" % (
            pair["ms"], pair["samples_executed"], pair["pairs_per_s"]))

    # ------------------------------------------------------------ serving
    serving = None
    if not args.no_serve and args.serve_queries > 0:
        serving = serving_leg(args, bc, gg)

    # ------------------------------------------------------- cpu baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        O = oracle.load()
        d1, e1, t1 = oracle_rate(O, g, host_src, comp_edges, args.cpu_seconds, 1)
        log("cpu oracle, 1 thread: %d sources in %.1f s -> %.4f GTEPS" % (d1, t1, e1 / t1 / 1e9))
        nt = max(1, min(args.cpu_threads, len(os.sched_getaffinity(0))))
        dn, en, tn = oracle_rate(O, g, host_src, comp_edges, args.cpu_seconds, nt)
        log("cpu oracle, %d threads: %d sources in %.1f s -> %.4f GTEPS" % (
            nt, dn, tn, en / tn / 1e9))
        cpu = {"value": en / tn / 1e9, "unit": "GTEPS", "cores": nt, "kind": "oracle",
               "sample": "first %d of the step's %d sources, fwd+bwd, summed, one source per "
                         "call on %d threads, %.1f s" % (dn, K, nt, tn),
               "single_thread": {"value": e1 / t1 / 1e9, "cores": 1,
                                 "sample": "first %d sources, %.1f s" % (d1, t1)}}

    res = {
        "metric": "sampled-source GTEPS (Brandes fwd+bwd), batched", "value": gteps,
        "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "BA n=2^20 m=5 (%d undirected edges), %d Philox-sampled sources "
                               "(seed %d), fwd+bwd, per-vertex dependency sum" % (
                                   g.m_undirected, K, args.seed),
                   "graph": args.graph, "n": g.n, "nnz": g.nnz, "sources": K,
                   "batch": st["batch_width"], "parallelism": "single GPU"},
        "per_source": per_source, "pair_leg": pair, "roofline": roofline, "cpu_baseline": cpu,
        "step_model": step_model, "serving": serving,
        "p99_query_ms": serving["p99_ms"] if serving else None,
        "kernels": [{"name": k["name"], "launches": k["launches"], "ms": k["ms"] / args.steps,
                     "algo_GBs": k["algo_bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] else 0.0}
                    for k in kern],
    }
    print(json.dumps(res), flush=True)
    G.close()


if __name__ == "__main__":
    main()
