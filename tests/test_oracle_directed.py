"""Pins for the oracle on directed graphs (Definition 1 over ordered pairs,
shortest paths following arc directions).

Expected values come from outside the oracle: brute-force enumeration of all
shortest directed paths with exact rationals, closed forms (directed paths,
cycles, stars), networkx's directed betweenness, and the undirected oracle on
bidirected graphs. Planted mistakes in the directed parts (path counts from
the wrong neighbour rows, a pair's second search over unreversed arcs, a
wrong transpose) must fail the pins.
"""
import os
import shutil
import subprocess
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


def random_digraph(seed, n=None):
    r = np.random.default_rng(seed)
    n = n or int(r.integers(5, 10))
    m = int(r.integers(n, 3 * n))
    return gg.from_arcs(n, r.integers(0, n, m), r.integers(0, n, m))


def check_against_brute(O_, g):
    b = Brute(g)
    bc = O_.bc_exact(g, directed=True)
    want = b.bc()
    if not all(close(bc[v], want[v]) for v in range(g.n)):
        return False
    for s in range(g.n):
        dist, (sm, se), de = O_.brandes(g, s, directed=True)
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
                y = O_.pair_dependency(g, s, t, directed=True)
                want = b.pair_dep(s, t)
                if not all(close(y[v], want[v]) for v in range(g.n)):
                    return False
    return True


@pytest.mark.parametrize("seed", range(30))
def test_brute_force_random_digraphs(seed):
    assert check_against_brute(O, random_digraph(500 + seed))


@pytest.mark.parametrize("n", [2, 3, 6, 20])
def test_directed_path(n):
    g = gg.directed_path(n)
    bc = O.bc_exact(g, directed=True)
    assert list(bc) == [i * (n - 1 - i) for i in range(n)]
    for s in range(n):
        dist, _, de = O.brandes(g, s, directed=True)
        for i in range(n):
            assert dist[i] == (i - s if i >= s else -1)
            assert de[i] == (n - 1 - i if i > s else 0)


@pytest.mark.parametrize("n", [3, 4, 7, 15])
def test_directed_cycle(n):
    # every ordered pair has one path; v lies strictly inside (n-1)(n-2)/2 of them
    assert np.all(O.bc_exact(gg.directed_cycle(n), directed=True) == (n - 1) * (n - 2) / 2)


def test_out_star_has_no_betweenness():
    assert np.all(O.bc_exact(gg.out_star(12), directed=True) == 0)


@pytest.mark.parametrize("seed", range(4))
def test_networkx_directed_betweenness(seed):
    g = gg.rmat_directed(7, 6, 0.57, 0.19, 0.19, seed=seed)
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.row))
    G.add_edges_from(zip(src.tolist(), g.col.tolist()))
    want = nx.betweenness_centrality(G, normalized=False)
    bc = O.bc_exact(g, directed=True)
    for v in range(g.n):
        assert close(bc[v], want[v], rel=1e-10, abs_=1e-9)


def test_bidirected_equals_undirected():
    g = gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=4)
    d = gg.bidirected(g)
    assert np.array_equal(O.bc_exact(d, directed=True), O.bc_exact(g))
    for s in (0, 7, 300):
        a, b = O.brandes(d, s, directed=True), O.brandes(g, s)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    assert np.array_equal(O.pair_dependency(d, 3, 400, directed=True),
                          O.pair_dependency(g, 3, 400))


def test_pair_dependencies_sum_to_bc():
    g = random_digraph(77, n=9)
    tot = np.zeros(g.n)
    for u in range(g.n):
        for v in range(g.n):
            if u != v:
                tot += O.pair_dependency(g, u, v, directed=True)
    assert np.allclose(tot, O.bc_exact(g, directed=True), rtol=1e-12, atol=1e-12)


def test_adaptive_samplers_replay_the_stream():
    g = gg.rmat_directed(8, 8, 0.57, 0.19, 0.19, seed=2)
    tg = gg.top_degree(g, 3)
    est, k, S, st = O.adaptive_source(g, tg, 1.5, 4, 400, directed=True)
    src = np.array([O.draw_source(4, j, g.n) for j in range(int(k.max()))], np.int32)
    full, _ = O.dependencies(g, src, full=True, total=False, directed=True)
    for i, t in enumerate(tg):
        assert S[i] == np.sum(full[:k[i], t]) or close(S[i], np.sum(full[:k[i], t]))
        assert est[i] == g.n * S[i] / k[i]
    est, k, S, st = O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.2, 1.0, 6, 3000, directed=True)
    y = np.zeros(len(tg))
    for j in range(int(k[0])):
        u, v = O.draw_pair(6, j, g.n)
        y[0] += O.pair_dependency(g, u, v, directed=True)[tg[0]]
    assert close(S[0], y[0])


# ------------------------------------------------------------ planted mistakes

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "oracle.h")
MUTANTS = {
    "counts_from_out_rows": ("    const int64_t *row = g->rrow;\n    const int32_t *col = g->rcol;",
                             "    const int64_t *row = g->row;\n    const int32_t *col = g->rcol;"),
    "pair_second_search_forward": ("graph_t r = {g->n, g->rrow, g->rcol, g->row, g->col};",
                                   "graph_t r = {g->n, g->row, g->col, g->rrow, g->rcol};"),
    "transpose_keeps_heads": ("tc[fill[col[e]]++] = (int32_t)u;", "tc[fill[col[e]]++] = col[e];"),
}


def pins_pass(O_):
    try:
        for seed in (500, 503, 511):
            if not check_against_brute(O_, random_digraph(seed)):
                return False
        if list(O_.bc_exact(gg.directed_cycle(7), directed=True)) != [15.0] * 7:
            return False
    except ValueError:
        return False
    return True


def test_unmodified_oracle_passes_the_directed_selection():
    assert pins_pass(O)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_directed_mistake_is_caught(tmp_path, name):
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
