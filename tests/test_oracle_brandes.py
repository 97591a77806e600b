"""Pins for the oracle's Brandes pass, exact BC and dependencies.

Each check comes from outside the oracle: brute-force enumeration of shortest
paths with exact rationals, closed forms, invariants of the definitions,
networkx and scipy, and binomial path counts on grids.
"""
import math
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


def from_nx(G):
    n = G.number_of_nodes()
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    if n == 0:
        return None
    return gg.from_edges(n, e[:, 0], e[:, 1])


def xval(m, e):
    """Exact rational value of an extended count m * 2^e."""
    return Fraction(float(m)) * (Fraction(2) ** int(e))


# ---------------------------------------------------------------- brute force

def check_against_brute(g):
    b = Brute(g)
    bc = O.bc_exact(g)
    want_bc = b.bc()
    for v in range(g.n):
        assert close(bc[v], want_bc[v]), (v, bc[v], want_bc[v])
    for s in range(g.n):
        dist, (sm, se), de = O.brandes(g, s)
        assert list(dist) == b.dist(s)
        sg = b.sigma(s)
        for v in range(g.n):
            assert xval(sm[v], se[v]) == sg[v]
        want = b.source_dep(s)
        for v in range(g.n):
            assert close(de[v], want[v]), (s, v, de[v], want[v])


def test_graph_atlas_all_small_graphs():
    """Every graph with at most 7 vertices (1253 graphs, connected or not)."""
    count = 0
    for G in nx.graph_atlas_g():
        g = from_nx(G)
        if g is None:
            continue
        check_against_brute(g)
        count += 1
    assert count == 1252


@pytest.mark.parametrize("seed", range(40))
def test_random_sparse_graphs_up_to_12(seed):
    r = np.random.default_rng(1000 + seed)
    n = int(r.integers(8, 13))
    m = int(r.integers(n - 2, int(1.6 * n)))
    G = nx.gnm_random_graph(n, m, seed=int(r.integers(1 << 30)))
    check_against_brute(from_nx(G))


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [2, 3, 5, 17, 64])
def test_path(n):
    bc = O.bc_exact(gg.path(n))
    for i in range(n):
        assert bc[i] == 2 * i * (n - 1 - i)


@pytest.mark.parametrize("n", [2, 3, 7, 40])
def test_path_source_dependency(n):
    g = gg.path(n)
    for s in range(n):
        _, _, de = O.brandes(g, s)
        for i in range(n):
            want = (n - 1 - i) if s < i else (i if s > i else 0)
            assert de[i] == want


@pytest.mark.parametrize("n", [3, 4, 10, 100])
def test_star(n):
    bc = O.bc_exact(gg.star(n))
    assert bc[0] == (n - 1) * (n - 2)
    assert np.all(bc[1:] == 0)


@pytest.mark.parametrize("n", [2, 3, 6, 25])
def test_complete(n):
    assert np.all(O.bc_exact(gg.complete(n)) == 0)


@pytest.mark.parametrize("n", [3, 5, 7, 9, 21, 101])
def test_odd_cycle(n):
    k = (n - 1) // 2
    assert np.all(O.bc_exact(gg.cycle(n)) == k * (k - 1))


@pytest.mark.parametrize("n", [4, 6, 8, 20, 100])
def test_even_cycle(n):
    k = n // 2
    assert np.allclose(O.bc_exact(gg.cycle(n)), (k - 1) ** 2, rtol=1e-13, atol=0)


@pytest.mark.parametrize("a,b", [(1, 3), (2, 3), (3, 5), (4, 4), (7, 2)])
def test_complete_bipartite(a, b):
    g = gg.complete_bipartite(a, b)
    bc = O.bc_exact(g)
    assert np.allclose(bc[:a], b * (b - 1) / a, rtol=1e-13)
    assert np.allclose(bc[a:], a * (a - 1) / b, rtol=1e-13)
    dist, (sm, se), _ = O.brandes(g, 0)
    for v in range(1, a):
        assert dist[v] == 2 and xval(sm[v], se[v]) == b
    for v in range(a, a + b):
        assert dist[v] == 1 and xval(sm[v], se[v]) == 1


def test_tree_counts_are_one():
    r = np.random.default_rng(5)
    n = 300
    parent = [int(r.integers(0, i)) for i in range(1, n)]
    g = gg.from_edges(n, np.arange(1, n), parent)
    for s in (0, 17, 299):
        _, (sm, se), _ = O.brandes(g, s)
        assert np.all(sm == 1.0) and np.all(se == 0)


# ------------------------------------------------------ sigma beyond 2^53

def test_grid_binomial_counts_beyond_2_53():
    x = y = 40
    g = gg.grid(x, y)
    dist, (sm, se), _ = O.brandes(g, 0)
    exceed = 0
    for i in range(x):
        for j in range(y):
            v = i * y + j
            want = math.comb(i + j, i)
            assert dist[v] == i + j
            got = xval(sm[v], se[v])
            if want < 2 ** 53:
                assert got == want
            else:
                exceed += 1
                assert abs(got - want) <= Fraction(want, 10 ** 12)
    assert exceed > 100


def test_grid_binomial_counts_beyond_fp64_range():
    x = y = 600
    g = gg.grid(x, y)
    dist, (sm, se), de = O.brandes(g, 0)
    assert np.all(np.isfinite(de))
    r = np.random.default_rng(3)
    pts = [(x - 1, y - 1), (x - 1, 0), (0, y - 1), (300, 300)] + \
          [tuple(map(int, r.integers(0, x, 2))) for _ in range(400)]
    beyond = 0
    for i, j in pts:
        v = i * y + j
        want = math.comb(i + j, i)
        got = xval(sm[v], se[v])
        assert dist[v] == i + j
        assert abs(got - want) <= Fraction(want, 10 ** 12), (i, j)
        beyond += want > 2 ** 1024
    assert beyond > 10


def test_grid_dependency_sum_invariant_large_counts():
    """The per-source invariant still holds when counts overflow FP64."""
    g = gg.grid(300, 300)
    dist, _, de = O.brandes(g, 0)
    want = float(np.sum(dist[dist > 0] - 1))
    assert close(de.sum(), want, rel=1e-9)


# ------------------------------------------------------------- invariants

def random_graph(seed, n=150, p=0.03):
    G = nx.gnp_random_graph(n, p, seed=seed)
    return from_nx(G)


@pytest.mark.parametrize("seed", range(5))
def test_source_dependency_sum_invariant(seed):
    g = random_graph(seed)
    for s in range(0, g.n, 7):
        dist, _, de = O.brandes(g, s)
        want = float(np.sum(dist[dist > 0] - 1))
        assert close(de.sum(), want, rel=1e-11)
        assert de[s] == 0
        assert np.all(de[dist < 0] == 0)


@pytest.mark.parametrize("seed", range(3))
def test_bc_sum_invariant(seed):
    g = random_graph(100 + seed, n=120, p=0.04)
    bc = O.bc_exact(g)
    tot = 0
    for s in range(g.n):
        dist, _, _ = O.brandes(g, s)
        tot += int(np.sum(dist[dist > 0] - 1))
    assert close(bc.sum(), tot, rel=1e-11)


# ------------------------------------------------------- third-party checks

@pytest.mark.parametrize("seed", range(4))
def test_networkx_betweenness(seed):
    """networkx counts unordered pairs on undirected graphs; BC here counts
    ordered pairs, so it is twice networkx's unnormalised value."""
    G = nx.gnp_random_graph(200, 0.025, seed=seed)
    g = from_nx(G)
    want = nx.betweenness_centrality(G, normalized=False)
    bc = O.bc_exact(g)
    for v in range(g.n):
        assert close(bc[v], 2 * want[v], rel=1e-10, abs_=1e-9)


def test_networkx_rmat_small():
    g = gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=11)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), g.degree())
    G.add_edges_from(zip(src.tolist(), g.col.tolist()))
    want = nx.betweenness_centrality(G, normalized=False)
    bc = O.bc_exact(g)
    for v in range(g.n):
        assert close(bc[v], 2 * want[v], rel=1e-10, abs_=1e-9)


def test_scipy_distances():
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    g = gg.rmat(10, 4, 0.57, 0.19, 0.19, seed=3)
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row), shape=(g.n, g.n))
    srcs = [0, 1, 5, 100, 777]
    D = shortest_path(a, unweighted=True, directed=False, indices=srcs)
    for i, s in enumerate(srcs):
        dist, _, _ = O.brandes(g, s)
        want = np.where(np.isinf(D[i]), -1, D[i]).astype(np.int64)
        assert np.array_equal(dist.astype(np.int64), want)


def test_dependencies_match_single_passes():
    g = random_graph(9)
    src = np.array([3, 3, 0, 149, 77], dtype=np.int32)
    full, tot = O.dependencies(g, src)
    acc = np.zeros(g.n)
    for i, s in enumerate(src):
        _, _, de = O.brandes(g, int(s))
        assert np.array_equal(full[i], de)
        acc += de
    assert np.array_equal(tot, acc)
    bc = O.bc_exact(g)
    _, tot_all = O.dependencies(g, np.arange(g.n, dtype=np.int32), full=False)
    assert np.array_equal(bc, tot_all)


def test_rejects_bad_arguments():
    g = gg.path(5)
    with pytest.raises(ValueError):
        O.brandes(g, 5)
    with pytest.raises(ValueError):
        O.dependencies(g, np.array([0, -1], dtype=np.int32))
