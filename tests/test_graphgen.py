"""Input generators used by the accuracy sweep: sizes, structure and the
clustering coefficient, checked against closed forms on the CPU."""
import numpy as np
import pytest

import graphgen as gg


def test_average_clustering_closed_forms():
    assert gg.average_clustering(gg.complete(7)) == pytest.approx(1.0)
    assert gg.average_clustering(gg.star(9)) == 0.0
    assert gg.average_clustering(gg.cycle(10)) == 0.0
    # K_{2,3}: no triangles
    assert gg.average_clustering(gg.complete_bipartite(2, 3)) == 0.0
    # a triangle with one pendant vertex: (1 + 1 + 1/3 + 0) / 4
    g = gg.from_edges(4, [0, 1, 0, 2], [1, 2, 2, 3])
    assert gg.average_clustering(g) == pytest.approx((1 + 1 + 1 / 3) / 4)


def test_small_world_lattice_and_rewiring():
    n, k = 200, 10
    lat = gg.small_world(n, k, 0.0, seed=1)
    assert lat.nnz == n * k
    assert (lat.degree() == k).all()
    # ring lattice: 3(k - 2) / (4(k - 1)) for every vertex
    assert gg.average_clustering(lat) == pytest.approx(3 * (k - 2) / (4 * (k - 1)))
    rw = gg.small_world(n, k, 0.2, seed=1)
    assert rw.nnz == n * k                      # rewiring keeps the edge count
    assert gg.average_clustering(rw) < gg.average_clustering(lat)
    assert np.array_equal(rw.col, gg.small_world(n, k, 0.2, seed=1).col)
    assert not np.array_equal(rw.col, gg.small_world(n, k, 0.2, seed=2).col)


def test_powerlaw_cluster_growth():
    n, m = 600, 3
    g = gg.powerlaw_cluster(n, m, 0.5, seed=4)
    assert g.nnz // 2 == m * (m + 1) // 2 + m * (n - m - 1)
    assert (g.degree() >= m).all()
    assert gg.largest_component(g).n == n     # growth keeps the graph connected
    # triad formation raises clustering over plain preferential attachment
    assert gg.average_clustering(g) > gg.average_clustering(
        gg.powerlaw_cluster(n, m, 0.0, seed=4)) + 0.1
    assert np.array_equal(g.col, gg.powerlaw_cluster(n, m, 0.5, seed=4).col)


def test_accuracy_stand_ins_match_the_dataset_table():
    import paper_1608_04472_amd.accuracy as acc
    o = acc.make_graph("oregon-like")
    f = acc.make_graph("facebook-like")
    assert o.n == 10670 and abs(o.nnz // 2 - 22002) / 22002 < 0.05
    assert abs(gg.average_clustering(o) - 0.2970) < 0.02
    assert f.n == 4039 and abs(f.nnz // 2 - 88234) / 88234 < 0.02
    assert abs(gg.average_clustering(f) - 0.6055) < 0.02


def test_top_targets_order():
    import paper_1608_04472_amd.accuracy as acc
    bcv = np.array([0.0, 3.0, 5.0, 5.0, 0.0, 1.0])
    assert acc.top_targets(bcv, 3).tolist() == [2, 3, 1]
    assert acc.top_targets(bcv, 10).tolist() == [2, 3, 1, 5]
