"""Pins for the oracle's work counters (the throughput metric's numerators).

oracle_source_work(s) -> (vertices reached from s, undirected edges of s's
component, shortest-path DAG edges from s: directed pairs (u, w) of adjacent
vertices with d(s,w) = d(s,u) + 1, i.e. the predecessor relation of
Definition 3). oracle_pair_work(u, v) -> undirected edges with an endpoint at
distance below d(u,v) from u (the edges a search from u that stops after the
destination's level has looked at; all of u's component when v is
unreachable).

Every expected value comes from outside the oracle: closed forms on paths,
stars, cycles, complete, bipartite and tree graphs, and distances from scipy's
breadth-first shortest paths with the edge counts taken by numpy.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle

O = oracle.load()


def scipy_dist(g, s):
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row), shape=(g.n, g.n))
    d = shortest_path(a, unweighted=True, directed=False, indices=[int(s)])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int64)


def edge_list(g):
    """Directed CSR entries (a, b) as two arrays."""
    a = np.repeat(np.arange(g.n), np.diff(g.row))
    return a, g.col.astype(np.int64)


def scipy_source_work(g, s):
    d = scipy_dist(g, s)
    a, b = edge_list(g)
    reached = int((d >= 0).sum())
    comp = int(((d[a] >= 0)).sum()) // 2
    dag = int(((d[a] >= 0) & (d[b] == d[a] + 1)).sum())
    return reached, comp, dag


def scipy_pair_work(g, u, v):
    d = scipy_dist(g, u)
    limit = d[v] if d[v] >= 0 else np.iinfo(np.int64).max
    a, b = edge_list(g)
    keep = a < b                              # each undirected edge once
    a, b = a[keep], b[keep]
    da, db = d[a], d[b]
    inside = (da >= 0) & (np.minimum(da, db) < limit)
    return int(inside.sum())


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [2, 3, 9, 40])
def test_path_source_work(n):
    g = gg.path(n)
    for s in range(n):
        assert O.source_work(g, s) == (n, n - 1, n - 1)


@pytest.mark.parametrize("n", [3, 10, 57])
def test_star_source_work(n):
    g = gg.star(n)
    for s in (0, 1, n - 1):
        assert O.source_work(g, s) == (n, n - 1, n - 1)


@pytest.mark.parametrize("n", [3, 5, 8, 11, 30])
def test_cycle_source_work(n):
    # even cycles: the antipode has two parents, every edge is a DAG edge;
    # odd cycles: the edge between the two farthest vertices joins one level
    g = gg.cycle(n)
    want_dag = n if n % 2 == 0 else n - 1
    for s in (0, n // 2):
        assert O.source_work(g, s) == (n, n, want_dag)


@pytest.mark.parametrize("n", [2, 5, 16])
def test_complete_source_work(n):
    g = gg.complete(n)
    assert O.source_work(g, 0) == (n, n * (n - 1) // 2, n - 1)


@pytest.mark.parametrize("a,b", [(1, 4), (3, 5), (6, 6)])
def test_bipartite_every_edge_is_a_dag_edge(a, b):
    # in a connected bipartite graph adjacent vertices differ by exactly one level
    g = gg.complete_bipartite(a, b)
    for s in (0, a):
        assert O.source_work(g, s) == (a + b, a * b, a * b)


@pytest.mark.parametrize("x,y", [(1, 7), (5, 9), (30, 30)])
def test_grid_every_edge_is_a_dag_edge(x, y):
    g = gg.grid(x, y)
    m = x * (y - 1) + y * (x - 1)
    for s in (0, x * y - 1, (x // 2) * y + y // 2):
        assert O.source_work(g, s) == (x * y, m, m)


def test_tree_dag_edges_are_reached_minus_one():
    r = np.random.default_rng(8)
    n = 400
    parent = [int(r.integers(0, i)) for i in range(1, n)]
    g = gg.from_edges(n, np.arange(1, n), parent)
    for s in (0, 123, 399):
        assert O.source_work(g, s) == (n, n - 1, n - 1)


def test_disconnected_counts_only_the_component():
    # a triangle, a path of 3 edges and an isolated vertex
    g = gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6])
    assert O.source_work(g, 0) == (3, 3, 2)
    assert O.source_work(g, 4) == (4, 3, 3)
    assert O.source_work(g, 7) == (1, 0, 0)


@pytest.mark.parametrize("n", [2, 7, 30])
def test_path_pair_work(n):
    g = gg.path(n)
    for u in range(n):
        for v in range(n):
            if u != v:
                k = abs(u - v)
                assert O.pair_work(g, u, v) == min(u, k) + min(k, n - 1 - u), (u, v)


@pytest.mark.parametrize("n", [3, 12])
def test_star_pair_work(n):
    g = gg.star(n)
    # from the centre or between two leaves every edge has an end below d(u,v);
    # from a leaf to the centre (d = 1) only the leaf's own edge does
    for u, v in ((0, 1), (1, 2), (n - 1, 1)):
        assert O.pair_work(g, u, v) == n - 1
    assert O.pair_work(g, 1, 0) == 1


def test_adjacent_pair_counts_the_start_row():
    g = gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=2)
    deg = g.degree()
    for u in gg.top_degree(g, 5):
        v = int(g.col[g.row[u]])
        assert O.pair_work(g, int(u), v) == deg[u]


def test_unreachable_destination_counts_the_whole_component():
    g = gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6])
    assert O.pair_work(g, 0, 5) == 3
    assert O.pair_work(g, 3, 7) == 3
    assert O.pair_work(g, 7, 0) == 0


# ------------------------------------------------------- scipy cross-checks

@pytest.mark.parametrize("seed", range(4))
def test_source_work_matches_scipy(seed):
    g = gg.rmat(10, 6, 0.57, 0.19, 0.19, seed=20 + seed)
    r = np.random.default_rng(seed)
    for s in list(r.integers(0, g.n, 12)) + list(gg.top_degree(g, 2)):
        assert O.source_work(g, int(s)) == scipy_source_work(g, s), s


@pytest.mark.parametrize("seed", range(4))
def test_pair_work_matches_scipy(seed):
    g = gg.er(500, 0.008, seed=30 + seed)
    r = np.random.default_rng(seed)
    for _ in range(25):
        u, v = (int(x) for x in r.choice(g.n, 2, replace=False))
        assert O.pair_work(g, u, v) == scipy_pair_work(g, u, v), (u, v)


def test_pair_work_bounded_by_the_component():
    g = gg.rmat(10, 6, 0.57, 0.19, 0.19, seed=4)
    r = np.random.default_rng(1)
    for _ in range(30):
        u, v = (int(x) for x in r.choice(g.n, 2, replace=False))
        _, comp, _ = O.source_work(g, u)
        assert O.pair_work(g, u, v) <= comp


# ----------------------------------------- the two-sided search's walk counts
#
# oracle_bidir_work(u, v) -> (vertices the search adds, arcs of the rows it
# reads), for the library's balanced two-sided search (side 0 from u over
# out-arcs, side 1 from v over in-arcs, the side with fewer frontier arcs
# expanding, ties to side 0; count pulls after each step; two sweeps after the
# meeting). Every expected value below was worked out by hand from those rules.

@pytest.mark.parametrize("n", [3, 5, 12])
def test_star_bidir_work(n):
    k = n - 1
    g = gg.star(n)
    # two leaves: each side walks its leaf's arc and the centre's row (count
    # pull), then each sweep reads the centre's row and its own leaf's arc
    assert O.bidir_work(g, 1, 2) == (2, 4 * k + 4)
    # centre and leaf, either order: one step from the leaf meets the centre
    assert O.bidir_work(g, 0, 1) == (1, 2 * k + 2)
    assert O.bidir_work(g, 1, 0) == (1, 2 * k + 2)


@pytest.mark.parametrize("n", [4, 6, 25])
def test_path_bidir_work(n):
    # ends of a path: side 0 steps first (tie), side 1 once (its frontier has
    # fewer arcs), then side 0 on every tie until it finds n-2; rows read:
    # 3 + 2(n-3) + 2(n-3) by side 0's steps and counts, 3 by side 1's, then
    # 2(n-2) + 2(n-3) + 1 and 3 by the sweeps: 8n - 12 arcs, n - 1 vertices
    g = gg.path(n)
    assert O.bidir_work(g, 0, n - 1) == (n - 1, 8 * n - 12)
    assert O.bidir_work(g, n - 1, 0) == (n - 1, 8 * n - 12)


@pytest.mark.parametrize("n", [2, 5, 30])
def test_directed_path_bidir_work(n):
    # side 0 walks the whole path on ties (n-1 steps of one arc, one in-arc
    # each for the counts), its sweep reads one in-arc and one out-arc per
    # level; backwards nothing is reachable
    g = gg.directed_path(n)
    assert O.bidir_work(g, 0, n - 1, directed=True) == (n - 1, 4 * (n - 1))
    assert O.bidir_work(g, n - 1, 0, directed=True) == (0, 0)


def test_unreachable_pair_bidir_work():
    # components {0,1,2} (a triangle) and {3,4,5,6} (a path), 7 isolated:
    # side 0 steps once (2 arcs, 2 found, counts 4), then side 1 three times
    # (2 + 3, 3 + 1, 1 arcs; 2 and 1 found), its last step adds nothing
    g = gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6])
    assert O.bidir_work(g, 0, 5) == (5, 16)
    assert O.bidir_work(g, 7, 0) == (0, 0)
    assert O.bidir_work(g, 0, 7) == (0, 0)


def test_meeting_step_counts_only_vertices_the_other_side_holds():
    # 0-1 adjacent, 0-2, 1-3, 2-4: the first step (side 0, a tie) adds 1 and 2
    # and meets at 1; only 1's row is read for the counts, and only 1's row
    # (not 2's) is marked in the sweep: 2 + 2 + 2 + 2 arcs
    g = gg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 4])
    assert O.bidir_work(g, 0, 1) == (2, 8)


def test_bidir_work_bounds():
    # every vertex is added at most once per side, and a side reads each of
    # its vertices' rows at most four times (its step, a count, a mark, a
    # sweep pull); a reachable pair adds at least d(u, v) vertices
    g = gg.rmat(10, 6, 0.57, 0.19, 0.19, seed=4)
    r = np.random.default_rng(2)
    deg = g.degree()
    for _ in range(40):
        u, v = (int(x) for x in r.choice(g.n, 2, replace=False))
        found, arcs = O.bidir_work(g, u, v)
        du, dv = scipy_dist(g, u), scipy_dist(g, v)
        assert found <= int((du >= 0).sum()) - 1 + int((dv >= 0).sum()) - 1
        assert arcs <= 4 * int(deg[du >= 0].sum() + deg[dv >= 0].sum())
        if du[v] > 0:
            assert found >= du[v]
        else:
            assert arcs <= int(deg[du >= 0].sum() + deg[dv >= 0].sum()) * 2


def test_ties_go_to_side_zero():
    # the path 0-3-1-2 and the pair (0, 1): side 0 steps first (1 arc against
    # 2) and finds 3; then 2 arcs against 2, a tie, so side 0 steps again and
    # meets at 1 (counts: 3's row, then 1's); side 1 never steps. The sweep
    # reads 1's and 3's rows at level 1, 3's and 0's at level 0: 2 vertices
    # found and 1 + 2 + 2 + 2 + 2 + 2 + 2 + 1 = 14 arcs (side 1 stepping on
    # the tie would add 2 and 3 instead: 3 vertices)
    g = gg.from_edges(4, [0, 3, 1], [3, 1, 2])
    assert O.bidir_work(g, 0, 1) == (2, 14)
