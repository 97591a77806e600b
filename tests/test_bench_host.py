"""Host-side helpers of bench.py (no GPU): the per-component edge count that
GTEPS divides by, the threaded oracle timing leg, and the traffic lookup."""
import importlib.util
import os
import sys

import numpy as np

import graphgen as gg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    argv = sys.argv
    sys.argv = ["bench.py"]
    try:
        spec.loader.exec_module(mod)
    finally:
        sys.argv = argv
    return mod


def test_component_edges_on_disconnected_graph():
    b = load_bench()
    # a triangle, a path of 3 edges and an isolated vertex
    g = gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6])
    assert b.component_edges(g).tolist() == [3, 3, 3, 3, 3, 3, 3, 0]


def test_oracle_rate_threads_cover_the_sources_once():
    b = load_bench()
    O = oracle.load()
    g = gg.config_graph("er2000")
    src = gg.philox_sources(1, 40, g.n)
    ce = b.component_edges(g)
    # a deadline of 0 stops after the first two sources have been taken
    d, e, _ = b.oracle_rate(O, g, src, ce, 0.0, 1)
    assert d == 2 and e == ce[src[:2]].sum()
    # a long deadline: every source exactly once, whatever the thread count
    for threads in (1, 4):
        d, e, _ = b.oracle_rate(O, g, src, ce, 1e9, threads)
        assert d == 40 and e == ce[src].sum()


def test_traffic_lookup_needs_a_matching_record():
    b = load_bench()
    assert b.measured_traffic("no_such_kernel", "ba1m-4096-b2048") is None
    assert b.measured_traffic("backward", "no_such_workload") is None


def test_pair_search_edges_equals_the_oracle_count():
    """bench.py's pair GTEPS counts edges with an endpoint below d(u,v) from
    distances; on random graphs (with isolated vertices) it must equal
    oracle_pair_work for every sampled pair, reachable or not."""
    b = load_bench()
    O = oracle.load()
    for g in (gg.rmat(9, 6, 0.57, 0.19, 0.19, seed=8), gg.er(400, 0.006, seed=2)):
        ea = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row))
        eb = g.col.astype(np.int64)
        r = np.random.default_rng(3)
        for _ in range(40):
            u, v = (int(x) for x in r.choice(g.n, 2, replace=False))
            dist = O.brandes(g, u)[0]
            assert b.pair_search_edges(dist, v, ea, eb) == O.pair_work(g, u, v), (u, v)


def test_cpu_info_fields():
    b = load_bench()
    info = b.cpu_info()
    assert info["nproc"] >= 1 and 1 <= info["usable"] <= info["nproc"]
