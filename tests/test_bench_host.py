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
