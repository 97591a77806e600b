"""Pins for the oracle on weighted graphs (Brandes' first step by Dijkstra's
algorithm, Section 3; Definitions 1-3 and Theorem 1 over weighted shortest
paths).

Expected values come from outside the oracle: brute-force enumeration of all
simple paths with their total weights and exact rationals, networkx's
weighted betweenness, the unweighted oracle (unit weights), invariance under
scaling every weight, and closed forms where a heavy edge leaves every
shortest path. Planted mistakes in the weighted code (a weight ignored, the
in-arc weights read for out-arcs, an unreached predecessor counted, the
source's own dependency kept, the ratio inverted, the transposed weights
misplaced) must fail the pins.
"""
import os
import shutil
import subprocess
from dataclasses import replace
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from bruteforce import Brute

O = oracle.load()


def close(a, b, rel=1e-12, abs_=1e-12):
    return abs(float(a) - float(b)) <= max(abs_, rel * abs(float(b)))


def xval(m, e):
    return Fraction(float(m)) * (Fraction(2) ** int(e))


def random_weighted(seed, directed, n=None, wmax=3):
    r = np.random.default_rng(seed)
    n = n or int(r.integers(5, 10))
    m = int(r.integers(n, 3 * n))
    a, b = r.integers(0, n, m), r.integers(0, n, m)
    g = gg.from_arcs(n, a, b) if directed else gg.from_edges(n, a, b)
    return gg.with_weights(g, wmax, seed=seed)


def check_against_brute(O_, g):
    d = g.directed
    b = Brute(g)
    bc = O_.bc_exact(g, directed=d)
    want = b.bc()
    if not all(close(bc[v], want[v]) for v in range(g.n)):
        return False
    for s in range(g.n):
        dist, (sm, se), de = O_.brandes(g, s, directed=d)
        if list(dist) != b.dist(s):
            return False
        sg = b.sigma(s)
        if any(xval(sm[v], se[v]) != sg[v] for v in range(g.n)):
            return False
        want = b.source_dep(s)
        if not all(close(de[v], want[v]) for v in range(g.n)):
            return False
        for t in range(g.n):
            if t != s:
                y = O_.pair_dependency(g, s, t, directed=d)
                want = b.pair_dep(s, t)
                if not all(close(y[v], want[v]) for v in range(g.n)):
                    return False
    return True


@pytest.mark.parametrize("directed", [False, True], ids=["undirected", "directed"])
@pytest.mark.parametrize("seed", range(20))
def test_brute_force_random_weighted(seed, directed):
    assert check_against_brute(O, random_weighted(900 + seed, directed))


def to_nx(g):
    G = nx.DiGraph() if g.directed else nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.row))
    for a, b, w in zip(src.tolist(), g.col.tolist(), g.w.tolist()):
        G.add_edge(a, b, weight=w)
    return G


@pytest.mark.parametrize("directed", [False, True], ids=["undirected", "directed"])
@pytest.mark.parametrize("seed", range(3))
def test_networkx_weighted_betweenness(seed, directed):
    base = gg.rmat_directed(7, 6, 0.57, 0.19, 0.19, seed=seed) if directed else \
        gg.rmat(7, 6, 0.57, 0.19, 0.19, seed=seed)
    g = gg.with_weights(base, 5, seed=seed)
    want = nx.betweenness_centrality(to_nx(g), normalized=False, weight="weight")
    bc = O.bc_exact(g, directed=directed)
    # networkx counts unordered pairs on an undirected graph
    f = 1 if directed else 2
    for v in range(g.n):
        assert close(bc[v], f * want[v], rel=1e-10, abs_=1e-9)


@pytest.mark.parametrize("directed", [False, True], ids=["undirected", "directed"])
def test_unit_weights_equal_the_unweighted_oracle(directed):
    base = gg.rmat_directed(9, 8, 0.57, 0.19, 0.19, seed=4) if directed else \
        gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=4)
    g = replace(base, w=np.ones(base.nnz, np.int32))
    assert np.array_equal(O.bc_exact(g, directed=directed), O.bc_exact(base, directed=directed))
    for s in (0, 9, 301):
        a, b = O.brandes(g, s, directed=directed), O.brandes(base, s, directed=directed)
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[1][0], b[1][0]) and np.array_equal(a[1][1], b[1][1])
        assert np.array_equal(a[2], b[2])
    assert np.array_equal(O.pair_dependency(g, 3, 400, directed=directed),
                          O.pair_dependency(base, 3, 400, directed=directed))


def test_scaled_weights_change_only_distances():
    g = gg.with_weights(gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=2), 6, seed=2)
    h = replace(g, w=(g.w * 7).astype(np.int32))
    assert np.array_equal(O.bc_exact(g), O.bc_exact(h))
    for s in (1, 77):
        a, b = O.brandes(g, s), O.brandes(h, s)
        assert np.array_equal(np.where(a[0] >= 0, a[0] * 7, -1), b[0])
        assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("n", [4, 7, 12])
def test_weighted_path_keeps_the_path_closed_form(n):
    # a path has one route per pair whatever its weights
    g = gg.with_weights(gg.path(n), 9, seed=n)
    assert list(O.bc_exact(g)) == [2 * i * (n - 1 - i) for i in range(n)]


@pytest.mark.parametrize("n", [5, 8, 11])
def test_heavy_edge_leaves_every_shortest_path(n):
    # a cycle whose closing edge weighs n is a path for shortest-path purposes
    g = gg.cycle(n)
    src = np.repeat(np.arange(n), np.diff(g.row))
    w = np.ones(g.nnz, np.int32)
    heavy = ((src == 0) & (g.col == n - 1)) | ((src == n - 1) & (g.col == 0))
    w[heavy] = n
    wg = replace(g, w=w)
    assert list(O.bc_exact(wg)) == [2 * i * (n - 1 - i) for i in range(n)]
    # at weight n - 1 the closing edge ties with the path from 0 to n-1
    w[heavy] = n - 1
    bc = O.bc_exact(replace(g, w=w))
    assert bc[1] < 2 * 1 * (n - 2)


def test_pair_dependencies_sum_to_bc():
    for directed in (False, True):
        g = random_weighted(77, directed, n=9)
        tot = np.zeros(g.n)
        for u in range(g.n):
            for v in range(g.n):
                if u != v:
                    tot += O.pair_dependency(g, u, v, directed=directed)
        assert np.allclose(tot, O.bc_exact(g, directed=directed), rtol=1e-12, atol=1e-12)


def test_samplers_replay_the_stream():
    g = gg.with_weights(gg.rmat(8, 8, 0.57, 0.19, 0.19, seed=2), 4, seed=3)
    tg = gg.top_degree(g, 3)
    est, k, S, st = O.adaptive_source(g, tg, 1.5, 4, 400)
    src = np.array([O.draw_source(4, j, g.n) for j in range(int(k.max()))], np.int32)
    full, _ = O.dependencies(g, src, full=True, total=False)
    for i, t in enumerate(tg):
        assert close(S[i], np.sum(full[:k[i], t]))
        assert est[i] == g.n * S[i] / k[i]
    est, k, S, st = O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.2, 1.0, 6, 3000)
    y = 0.0
    for j in range(int(k[0])):
        u, v = O.draw_pair(6, j, g.n)
        y += O.pair_dependency(g, u, v)[tg[0]]
    assert close(S[0], y)


def test_weight_validation():
    g = gg.with_weights(gg.path(5), 3, seed=1)
    bad = replace(g, w=np.where(np.arange(g.nnz) == 2, 0, g.w).astype(np.int32))
    with pytest.raises(ValueError):
        O.bc_exact(bad)
    # an undirected edge whose two arcs disagree
    asym = g.w.copy()
    asym[0] += 1
    with pytest.raises(ValueError):
        O.bc_exact(replace(g, w=asym))
    # max weight * (n - 1) must stay below 2^30
    with pytest.raises(ValueError):
        O.bc_exact(replace(g, w=np.full(g.nnz, 1 << 28, np.int32)))


# ------------------------------------------------------------ planted mistakes

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "oracle.h")
MUTANTS = {
    "dijkstra_ignores_weight": ("const int32_t through = p->dist[u] + g->wt[e];",
                                "const int32_t through = p->dist[u] + 1;"),
    "successor_in_arc_weights": ("if (p->dist[v] + g->wt[e] == p->dist[t])",
                                 "if (p->dist[v] + g->rwt[e] == p->dist[t])"),
    "predecessor_not_on_a_shortest_path": (
        "if (p->dist[u] >= 0 && p->dist[u] + g->rwt[e] == p->dist[w])",
        "if (p->dist[u] >= 0 && p->dist[u] < p->dist[w])"),
    "weighted_source_kept": ("for (int64_t i = p->reached - 1; i > 0; --i) {",
                             "for (int64_t i = p->reached - 1; i >= 0; --i) {"),
    "weighted_ratio_inverted": ("sum += xnum_div(p->sig[v], p->sig[t]) * (1.0 + p->delta[t]);",
                                "sum += xnum_div(p->sig[t], p->sig[v]) * (1.0 + p->delta[t]);"),
    "transposed_weights_misplaced": ("tw[next[col[e]]++] = wt[e];",
                                     "tw[next[col[e]]++] = wt[row[u]];"),
}


def pins_pass(O_):
    try:
        for seed in (900, 905, 911):
            for directed in (False, True):
                if not check_against_brute(O_, random_weighted(seed, directed)):
                    return False
        g = gg.with_weights(gg.rmat_directed(7, 6, 0.57, 0.19, 0.19, seed=1), 5, seed=1)
        want = nx.betweenness_centrality(to_nx(g), normalized=False, weight="weight")
        bc = O_.bc_exact(g, directed=True)
        if not all(close(bc[v], want[v], rel=1e-10, abs_=1e-9) for v in range(g.n)):
            return False
    except ValueError:
        return False
    return True


def test_unmodified_oracle_passes_the_weighted_selection():
    assert pins_pass(O)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_weighted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    d = tmp_path / name
    d.mkdir()
    shutil.copy(HDR, d / "oracle.h")
    (d / "oracle.c").write_text(src.replace(old, new))
    out = str(d / "lib.so")
    subprocess.check_call(["gcc"] + oracle.CFLAGS + [str(d / "oracle.c"), "-o", out, "-lm"])
    assert not pins_pass(oracle.load(out))
