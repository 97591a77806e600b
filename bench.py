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
  pair_leg    adaptive pair sampling (eps = 0.05, 32 top-degree targets), with
              pair-search GTEPS and its dominant kernel's roofline
  roofline    the dominant kernel against the 8 TB/s HBM peak
  cpu_baseline the CPU oracle on a bounded sample of the same sources
  legs        the other workloads: C1 (ER n = 2000: exact BC and the three
              samplers), C2 (R-MAT scale 16: 64 degree-percentile targets,
              c = 5, 256 per round), C4 (2048^2 grid, 5 % of edges removed, 1024
              sources), w (the C3 graph with arc weights in [1, 100], 1024
              sources) and C5 (serving a prefix of the 20,000-query stream)
The graph's plan comes from the autotuner (bc_graph_tune) unless --schedule
names one; it is part of the printed config.
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
# the dominant kernel's source and the host code that launches it
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


def pair_search_edges(dist, v, ea, eb):
    """Undirected edges with an endpoint at distance < d(u, v) from u, the
    edges a search from u that stops after v's level has looked at (all of u's
    component when v is unreachable). dist: distances from u (-1 unreached);
    ea, eb: the CSR's directed entries."""
    import numpy as np
    lim = dist[v] if dist[v] >= 0 else np.iinfo(np.int64).max
    da = dist[ea].astype(np.int64)
    db = dist[eb].astype(np.int64)
    keep = ea < eb
    lo = np.minimum(da[keep], db[keep])
    return int(((da[keep] >= 0) & (lo < lim)).sum())


def cpu_info():
    """Model name, logical CPUs of the host and CPUs this process may use."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "usable": len(os.sched_getaffinity(0))}


def sampler_gteps(bc, G, gg, comp_edges, seed, executed, pairs):
    """Undirected edges searched by a sampler's executed samples: for sources,
    each source's component (Graph500 convention); pairs are not counted here."""
    import numpy as np
    src = gg.philox_sources(seed, int(executed), G.n)
    return float(np.asarray(comp_edges)[src].sum())


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
    S.set_lanes(args.serve_lanes)       # before admission: widths fit one workspace per lane
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
        "queries": N, "arrival_rate_qps": args.serve_rate, "lanes": args.serve_lanes,
        "achieved_qps": N / makespan, "makespan_s": makespan,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()), "rounds": st["rounds"],
        "samples_executed": st["samples_executed"], "samples_used": st["samples_used"],
        "batch_fill": st["samples_executed"] / max(1, args.serve_batch * st["rounds"]),
        "capped": int(sum(r["status"] == bc.BC_CAPPED for r in res)),
        "capped_fraction": float(np.mean([r["status"] == bc.BC_CAPPED for r in res])),
        "offered_qps": N / max(1e-9, max(q["arrival"] for q in qs)),
        "split_rounds": st["split_rounds"], "budget_bytes": st["budget_bytes"],
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
    log("serving (%d lanes): p50 %.1f ms, p99 %.1f ms, %.1f q/s achieved over %.1f s, %d rounds, "
        "capped %.2f" % (args.serve_lanes, out["p50_ms"], out["p99_ms"], out["achieved_qps"],
                         makespan, st["rounds"], out["capped_fraction"]))
    return out


def c1_leg(args, bc, gg, dev):
    """ER n = 2000 (graph seed 1): exact BC; source sampling c = 5, pair sampling
    eps = 0.1 and Algorithm 1 as printed (c = 1) for the 16 highest-degree
    vertices, seed 1."""
    import torch
    g = gg.config_graph("er2000")
    ce = component_edges(g)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_TUNED)
    out = {"workload": "ER n=2000 p=8/1999 (seed 1), %d undirected edges" % g.m_undirected}
    bc.exact(G)                                     # tunes, warms
    torch.cuda.synchronize()
    t = time.perf_counter()
    bc.exact(G)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    out["exact"] = {"ms": 1e3 * dt, "gteps": float(ce.sum()) / dt / 1e9}
    tg = torch.from_numpy(gg.top_degree(g, 16)).to(dev)
    for name, call in (("source_c5", lambda: bc.adaptive_source(G, tg, 5.0, 1, g.n)),
                       ("pair_eps0.1", lambda: bc.adaptive_pair(G, tg, bc.BC_PAIR_EPS, 0.1, 1.0,
                                                                1, 1 << 20)),
                       ("pair_alg1_c1", lambda: bc.adaptive_pair(G, tg, bc.BC_PAIR_ALG1, 0.1, 1.0,
                                                                 1, 1 << 20))):
        torch.cuda.synchronize()
        t = time.perf_counter()
        est, k, S, st = call()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        ex = G.stats()["samples_executed"]
        kk = k.cpu().numpy()
        rec = {"ms": 1e3 * dt, "samples_executed": int(ex), "samples_used": int(kk.max()),
               "capped": int((st.cpu().numpy() == bc.BC_CAPPED).sum()),
               "samples_per_s": ex / dt, "bottom_up": G.stats()["bottom_up"]}
        if name.startswith("source"):
            rec["gteps"] = sampler_gteps(bc, G, gg, ce, 1, ex, False) / dt / 1e9
        out[name] = rec
    out["plan"] = G.plan()
    G.close()
    log("C1: exact %.1f ms; source %.1f ms; pair eps %.1f ms; alg1 %.1f ms (%d pairs)" % (
        out["exact"]["ms"], out["source_c5"]["ms"], out["pair_eps0.1"]["ms"],
        out["pair_alg1_c1"]["ms"], out["pair_alg1_c1"]["samples_executed"]))
    return out


def c2_leg(args, bc, gg, dev):
    """R-MAT scale 16 (graph seed 2): adaptive source sampling for 64 targets at
    degree percentiles among degree >= 2 vertices, c = 5, 256 samples per round,
    seed 2, k_max = n."""
    import torch
    g = gg.config_graph("rmat16")
    ce = component_edges(g)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_TUNED, 256)
    tg = torch.from_numpy(gg.degree_percentile_targets(g, 64)).to(dev)
    bc.adaptive_source(G, tg[:2].contiguous(), 5.0, 2, 300)          # tunes, warms
    torch.cuda.synchronize()
    t = time.perf_counter()
    est, k, S, st = bc.adaptive_source(G, tg, 5.0, 2, g.n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ex = G.stats()["samples_executed"]
    kk = k.cpu().numpy()
    stt = st.cpu().numpy()
    out = {"workload": "R-MAT scale 16 ef 16 (seed 2), %d undirected edges; 64 degree-percentile "
                       "targets, c=5, 256 per round, k_max=n" % g.m_undirected,
           "ms": 1e3 * dt, "samples_executed": int(ex), "samples_used_sum": int(kk.sum()),
           "samples_used_max": int(kk.max()), "rounds": int(G.stats()["batches"]),
           "capped": int((stt == bc.BC_CAPPED).sum()), "done": int((stt == bc.BC_DONE).sum()),
           "gteps": sampler_gteps(bc, G, gg, ce, 2, ex, False) / dt / 1e9, "plan": G.plan(),
           "round_bottom_up": G.stats()["bottom_up"]}
    G.close()
    log("C2: %.1f ms, %d sources executed, %d capped, %.2f GTEPS" % (
        out["ms"], ex, out["capped"], out["gteps"]))
    return out


def schedule_id(bc, name):
    return {"tuned": bc.BC_SCHED_TUNED, "auto": bc.BC_SCHED_AUTO, "wave": bc.BC_SCHED_BATCHED,
            "pair": bc.BC_SCHED_THREADED, "wg": bc.BC_SCHED_WORKGROUP}[name]


def c4_leg(args, bc, gg, dev):
    """2048^2 grid, 5 % of edges removed (seed 3), largest component: 1024
    sources (seed 3), fwd+bwd, per-vertex sum; one step after a warm-up, under
    the tuned plan unless --c4-schedule names one."""
    import torch
    t0 = time.time()
    g = gg.config_graph("grid2048")
    ce = component_edges(g)
    G = bc.Graph(g.row, g.col)
    G.configure(schedule_id(bc, args.c4_schedule), args.c4_batch)
    tune_s = 0.0
    if args.c4_schedule == "tuned":
        t = time.time()
        G.tune()
        tune_s = time.time() - t
    K = 1024
    srcs = torch.from_numpy(gg.philox_sources(3, K, g.n)).to(dev)
    out_t = torch.empty(g.n, dtype=torch.float64, device=dev)
    # the tuner's released buffers sit in torch's cache, which the device's
    # free-memory count (by which a plan is sized) does not see
    torch.cuda.empty_cache()
    bc.bc_dependencies(G, srcs, bc.BC_OUT_SUM, out_t)   # warm-up: the same step
    torch.cuda.synchronize()
    G.profile(True)
    t = time.perf_counter()
    bc.bc_dependencies(G, srcs, bc.BC_OUT_SUM, out_t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    kern = G.profile_read()
    G.profile(False)
    st = G.stats()
    edges = float(ce[srcs.cpu().numpy()].sum())
    out = {"workload": "2048^2 grid, 5%% of edges removed (seed 3), n=%d, %d undirected edges; "
                       "1024 sources (seed 3), fwd+bwd, sum" % (g.n, g.m_undirected),
           "ms_per_step": 1e3 * dt, "gteps": edges / dt / 1e9, "levels": int(st["levels"]),
           "batch": int(st["batch_width"]), "extended": int(st["extended"]),
           "launches": int(sum(k["launches"] for k in kern)), "plan": G.plan(),
           "kernels": {k["name"]: {"ms": k["ms"], "launches": k["launches"]}
                       for k in kern if k["launches"]},
           "tune_s": tune_s, "setup_s": time.time() - t0 - dt}
    G.close()
    log("C4: %.0f ms/step, %.2f GTEPS, %d levels, batch %d, %d hot launches, plan %s" % (
        out["ms_per_step"], out["gteps"], out["levels"], out["batch"], out["launches"],
        out["plan"]))
    return out


def weighted_leg(args, bc, gg, dev):
    """The C3 graph (BA, n = 2^20, m = 5, seed 7) with integer arc weights
    drawn uniformly from [1, 100] (seed 7, one per edge): 1024 sources (seed 7),
    fwd+bwd, per-vertex sum; one step after a warm-up. GTEPS counts each
    source's component edges once, as the unweighted legs do."""
    import torch
    t0 = time.time()
    g = gg.with_weights(gg.config_graph("ba1m"), 100, seed=7)
    ce = component_edges(g)
    G = bc.Graph(g.row, g.col, weights=g.w)
    K = 1024
    srcs = torch.from_numpy(gg.philox_sources(7, K, g.n)).to(dev)
    out_t = torch.empty(g.n, dtype=torch.float64, device=dev)
    bc.bc_dependencies(G, srcs, bc.BC_OUT_SUM, out_t)   # warm-up: the same step
    torch.cuda.synchronize()
    G.profile(True)
    t = time.perf_counter()
    bc.bc_dependencies(G, srcs, bc.BC_OUT_SUM, out_t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    kern = G.profile_read()
    G.profile(False)
    st = G.stats()
    edges = float(ce[srcs.cpu().numpy()].sum())
    by = {k["name"]: k for k in kern}
    dom = max(kern, key=lambda x: x["ms"])
    ach = dom["algo_bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    relax = by["w_search"]["units_a"]
    out = {"workload": "BA n=2^20, m=5 (seed 7), arc weights uniform in [1, 100] (seed 7); "
                       "1024 sources (seed 7), fwd+bwd, sum",
           "ms_per_step": 1e3 * dt, "gteps": edges / dt / 1e9,
           "rounds_counts": int(st["levels"]), "batch": int(st["batch_width"]),
           "search_launches": int(by["w_search"]["launches"]),
           "relaxations_per_arc": relax / (2.0 * edges) if edges else None,
           "launches": int(sum(k["launches"] for k in kern)),
           "kernels": {k["name"]: {"ms": k["ms"], "launches": k["launches"]}
                       for k in kern if k["launches"]},
           "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS},
           "setup_s": time.time() - t0 - dt}
    G.close()
    log("weighted: %.0f ms/step, %.2f GTEPS, batch %d, %d search rounds, %.2f relaxations "
        "per arc, dominant %s %.1f GB/s" % (out["ms_per_step"], out["gteps"], out["batch"],
                                             out["search_launches"], out["relaxations_per_arc"]
                                             or 0.0, dom["name"], ach))
    return out


def pair_leg(args, bc, gg, G, g, dev):
    """Adaptive pair sampling (eps, the top-degree targets, seed 7): time,
    samples, pair-search GTEPS (edges with an endpoint below d(u,v), measured on
    an evenly spaced sample of the executed pairs and scaled to all of them) and
    the dominant kernel's roofline."""
    import numpy as np
    import torch
    targets = torch.from_numpy(gg.top_degree(g, args.pair_targets)).to(dev)
    search = {"auto": bc.BC_PAIR_SEARCH_AUTO, "one": bc.BC_PAIR_SEARCH_ONE_SIDED,
              "bidir": bc.BC_PAIR_SEARCH_BIDIRECTIONAL}

    def run(mode):
        G.configure(bc.BC_SCHED_TUNED, 0, 0.0, 0, 0, args.pair_sampler_batch, search[mode])
        G.plan()                      # the tuned plan from the cache, outside the timing
        # warm-up: the same run once, so its workspace is in place before timing
        bc.adaptive_pair(G, targets, bc.BC_PAIR_EPS, args.pair_eps, 1.0, args.seed, 1 << 20)
        torch.cuda.synchronize()
        G.profile(True)
        t = time.perf_counter()
        res = bc.adaptive_pair(G, targets, bc.BC_PAIR_EPS, args.pair_eps, 1.0, args.seed, 1 << 20)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        kern = G.profile_read()
        G.profile(False)
        return res, el, kern, G.stats()

    one = None
    if args.pair_search == "auto":
        # the one-sided search on the same stream, for comparison
        (_, k1, _, _), t1, _, st1 = run("one")
        one = {"ms": 1e3 * t1, "pairs_per_s": int(st1["samples_executed"]) / t1,
               "samples_executed": int(st1["samples_executed"])}
    (est, k, S, stt), pt, kern, pst = run(args.pair_search)
    G.configure(bc.BC_SCHED_TUNED, 0, 0.0, 0, 0, 0, 0)
    ex = int(pst["samples_executed"])
    kk = k.cpu().numpy()
    if one is not None:
        assert np.array_equal(kk, k1.cpu().numpy()), "pair searches disagree on samples used"
    # pair-search edges on a sample of the executed pairs: distances from u by
    # the library (pinned to the oracle), edges counted on the host
    m = min(args.pair_work_sample, ex)
    js = np.unique(np.linspace(0, ex - 1, m).astype(np.int64))
    us = torch.empty(ex, dtype=torch.int32, device=dev)
    vs = torch.empty(ex, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, args.seed, 0, ex, us, vs)
    su = us[torch.from_numpy(js).to(dev)].contiguous()
    sv = vs[torch.from_numpy(js).to(dev)].cpu().numpy()
    _, dist, _ = bc.dependencies(G, su, bc.BC_OUT_FULL, dist=True)
    dist = dist.cpu().numpy()
    ea = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row))
    eb = g.col.astype(np.int64)
    work = [pair_search_edges(dist[i], int(sv[i]), ea, eb) for i in range(len(js))]
    mean_work = float(np.mean(work))
    dom = max(kern, key=lambda x: x["ms"])
    ach = dom["algo_bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    bi = next(x for x in kern if x["name"] == "bidir_pair")
    out = {"targets": args.pair_targets, "eps": args.pair_eps, "ms": 1e3 * pt,
           "pair_search": {1: "one-sided", 2: "bidirectional"}.get(int(pst["pair_search"]), "?"),
           "one_sided": one,
           "bidir_arcs_walked_per_pair": bi["units_b"] / ex if bi["launches"] else None,
           "bidir_vertices_found_per_pair": bi["units_a"] / ex if bi["launches"] else None,
           "samples_executed": ex, "samples_used_max": int(kk.max()),
           "samples_used_min": int(kk.min()), "pairs_per_s": ex / pt,
           "rounds": int(pst["batches"]), "capped": int((stt.cpu().numpy() == bc.BC_CAPPED).sum()),
           "pair_search_edges_mean": mean_work,
           "pair_work_sample": "%d of the %d executed pairs, evenly spaced in draw order" % (
               len(js), ex),
           "gteps": mean_work * ex / pt / 1e9,
           "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": ach,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}}
    log("pair leg (%s): %.1f ms, %d pairs executed (%.0f pairs/s), %.2f GTEPS (one-sided "
        "pair-search edges)" % (out["pair_search"], out["ms"], ex, out["pairs_per_s"],
                                out["gteps"]))
    if bi["launches"]:
        log("  bidir_pair: %d launches %.1f ms, %.0f arcs walked and %.0f vertices found per pair"
            " (one-sided search: %.0f edges), %.1f GB/s algorithmic" % (
                bi["launches"], bi["ms"], out["bidir_arcs_walked_per_pair"],
                out["bidir_vertices_found_per_pair"], mean_work,
                bi["algo_bytes"] / (bi["ms"] * 1e-3) / 1e9 if bi["ms"] > 0 else 0.0))
    if one is not None:
        log("  one-sided on the same stream: %.1f ms (%.0f pairs/s)" % (one["ms"],
                                                                      one["pairs_per_s"]))
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
    ap.add_argument("--schedule", default="tuned", choices=["tuned", "auto", "wave", "pair", "wg"])
    ap.add_argument("--bottom-up", type=float, default=0.0)
    ap.add_argument("--level-loop", type=int, default=0,
                    help="pair engine: 1 persistent level loops, else one launch per level phase")
    ap.add_argument("--per-source", type=int, default=16, help="sources for the per-source leg")
    ap.add_argument("--pair-targets", type=int, default=32)
    ap.add_argument("--pair-eps", type=float, default=0.05)
    ap.add_argument("--pair-work-sample", type=int, default=64,
                    help="executed pairs whose search edges are counted for the pair GTEPS")
    ap.add_argument("--pair-sampler-batch", type=int, default=0,
                    help="samples per pair-sampler round (0 = the library's default)")
    ap.add_argument("--pair-search", default="auto", choices=["auto", "one", "bidir"],
                    help="pair samples' search; auto also times the one-sided one")
    ap.add_argument("--no-pair", action="store_true")
    ap.add_argument("--legs", default="c1,c2,c4,w,c5",
                    help="other workloads to measure (comma list of c1, c2, c4, c5; '' = none)")
    ap.add_argument("--c4-batch", type=int, default=0,
                    help="C4 batch width (0: the schedule's own)")
    ap.add_argument("--c4-schedule", default="tuned",
                    choices=["tuned", "auto", "wave", "pair", "wg"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="threads for the all-cores oracle run (capped by the CPUs this "
                         "process may use)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-graphs", type=int, default=200)
    ap.add_argument("--serve-queries", type=int, default=2000,
                    help="prefix of the 20,000-query stream to serve (the whole stream "
                         "exceeds one GPU's capacity)")
    ap.add_argument("--serve-rate", type=float, default=500.0)
    ap.add_argument("--serve-budget-gib", type=int, default=128)
    ap.add_argument("--serve-lanes", type=int, default=4,
                    help="serving rounds of this many graphs at once (own streams)")
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
    sched = schedule_id(bc, args.schedule)
    G.configure(sched, args.batch, args.bottom_up, 0, args.level_loop)
    if sched == bc.BC_SCHED_TUNED:
        t = time.time()
        plan = G.tune()
        log("tuned in %.1fs: %s" % (time.time() - t, plan))
    plan = G.plan()

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
    fwd = next(k for k in kern if k["name"] == "pair_forward")
    csr_bytes = 8 * (g.n + 1) + 4 * g.nnz
    batches = -(-K // st["batch_width"])
    reach = sig["units_a"] + fwd["units_a"] + K * args.steps   # level-0 pairs are the sources
    dag = sig["units_b"] + fwd["units_b"]
    step_bytes = (2 * csr_bytes * batches * args.steps + 32 * reach + 16 * dag) / args.steps
    step_model = {"algo_bytes": step_bytes, "GBs": step_bytes / (ms * 1e-3) / 1e9,
                  "frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                  "reached_pairs": reach / args.steps, "dag_edge_pairs": dag / args.steps}
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
        pair = pair_leg(args, bc, gg, G, g, dev)
    G.close()

    # ------------------------------------------------------ other workloads
    legs = {}
    want = [x for x in args.legs.split(",") if x]
    for name, fn in (("c1", c1_leg), ("c2", c2_leg), ("c4", c4_leg), ("w", weighted_leg)):
        if name in want:
            # the library sizes its buffers from the device's free memory:
            # hand back what torch's allocator cached for the previous leg
            torch.cuda.empty_cache()
            legs[name] = fn(args, bc, gg, dev)
    serving = None
    if "c5" in want and not args.no_serve and args.serve_queries > 0:
        serving = serving_leg(args, bc, gg)

    # ------------------------------------------------------- cpu baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        O = oracle.load()
        d1, e1, t1 = oracle_rate(O, g, host_src, comp_edges, args.cpu_seconds, 1)
        log("cpu oracle, 1 thread: %d sources in %.1f s -> %.4f GTEPS" % (d1, t1, e1 / t1 / 1e9))
        info = cpu_info()
        nt = max(1, min(args.cpu_threads, info["usable"]))
        dn, en, tn = oracle_rate(O, g, host_src, comp_edges, args.cpu_seconds, nt)
        log("cpu oracle, %d threads: %d sources in %.1f s -> %.4f GTEPS" % (
            nt, dn, tn, en / tn / 1e9))
        cpu = {"value": en / tn / 1e9, "unit": "GTEPS", "cores": nt, "kind": "oracle",
               "sample": "first %d of the step's %d sources, fwd+bwd, summed, one source per "
                         "call on %d threads, %.1f s" % (dn, K, nt, tn),
               "cpu_model": info["model"], "nproc": info["nproc"],
               "usable_cpus": info["usable"],
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
                   "batch": st["batch_width"], "plan": plan, "parallelism": "single GPU"},
        "per_source": per_source, "pair_leg": pair, "roofline": roofline, "cpu_baseline": cpu,
        "step_model": step_model, "legs": legs, "serving": serving,
        "p99_query_ms": serving["p99_ms"] if serving else None,
        "kernels": [{"name": k["name"], "launches": k["launches"], "ms": k["ms"] / args.steps,
                     "algo_GBs": k["algo_bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] else 0.0}
                    for k in kern],
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
