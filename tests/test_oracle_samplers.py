"""Pins for the oracle's Philox stream, draws, pair dependencies and samplers.

The sample stream is checked against numpy's Philox4x64-10 (independent code).
The loops are checked on graphs where the per-sample value is known in closed
form, so the stopping sample can be worked out from the draw stream alone.
"""
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from bruteforce import Brute

O = oracle.load()
U64 = np.uint64


def numpy_block(seed, stream, j):
    """Philox4x64-10 block j under key (seed, stream), from numpy.
    numpy emits block c+1 first when its counter is c."""
    c = (j - 1) % (1 << 256)
    ctr = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=U64)
    bg = np.random.Philox(key=np.array([seed, stream], dtype=U64), counter=ctr)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("seed,stream,j", [(0, 0, 0), (7, 0, 0), (7, 0, 1), (7, 0, 4095),
                                           (1, 1, 12345), ((1 << 64) - 1, 3, 99),
                                           (0xDEADBEEF, 1, (1 << 40) + 3)])
def test_philox_matches_numpy(seed, stream, j):
    got = O.philox([j, 0, 0, 0], [seed, stream])
    assert [int(x) for x in got] == numpy_block(seed, stream, j)


def test_philox_full_counter_words():
    ctr = [0x0123456789ABCDEF, 0xFEDCBA9876543210, 7, 1 << 63]
    c = sum(w << (64 * i) for i, w in enumerate(ctr))
    got = O.philox(ctr, [42, 43])
    assert [int(x) for x in got] == numpy_block(42, 43, c)


@pytest.mark.parametrize("n", [2, 3, 1000, (1 << 20), 4194274])
def test_draws_follow_published_map(n):
    for seed in (1, 7):
        for j in (0, 1, 2, 1000):
            w = numpy_block(seed, 0, j)
            assert O.draw_source(seed, j, n) == (w[0] * n) >> 64
            w = numpy_block(seed, 1, j)
            u = (w[0] * n) >> 64
            v = (w[1] * (n - 1)) >> 64
            v += v >= u
            assert O.draw_pair(seed, j, n) == (u, v)


def test_fixed_source_list_generator_agrees():
    """graphgen's source lists use the same map through numpy's Philox."""
    src = gg.philox_sources(7, 64, 1 << 20)
    assert [O.draw_source(7, j, 1 << 20) for j in range(64)] == src.tolist()


def test_pair_draws_cover_ordered_pairs_uniformly():
    n = 5
    counts = np.zeros((n, n))
    N = 40000
    for j in range(N):
        u, v = O.draw_pair(3, j, n)
        assert u != v
        counts[u, v] += 1
    off = counts[~np.eye(n, dtype=bool)]
    exp = N / (n * (n - 1))
    chi2 = float(np.sum((off - exp) ** 2 / exp))
    assert chi2 < 60.0   # 19 degrees of freedom; p < 1e-5 beyond this


# ----------------------------------------------------------- pair dependency

def check_pairs_brute(g):
    b = Brute(g)
    for u in range(g.n):
        for v in range(g.n):
            if u == v:
                continue
            y = O.pair_dependency(g, u, v)
            want = b.pair_dep(u, v)
            for t in range(g.n):
                assert abs(y[t] - float(want[t])) <= 1e-15 * max(1.0, float(want[t])), (u, v, t)


def test_pair_dependency_bruteforce_atlas_sample():
    atlas = nx.graph_atlas_g()
    for G in atlas[1::9]:
        if G.number_of_nodes() < 2:
            continue
        e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
        check_pairs_brute(gg.from_edges(G.number_of_nodes(), e[:, 0], e[:, 1]))


@pytest.mark.parametrize("seed", range(6))
def test_pair_dependency_bruteforce_random(seed):
    G = nx.gnm_random_graph(10, 14, seed=seed)
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    check_pairs_brute(gg.from_edges(10, e[:, 0], e[:, 1]))


@pytest.mark.parametrize("seed", range(3))
def test_pair_dependencies_sum_to_bc(seed):
    """Summing sigma_uv(t)/sigma_uv over all ordered pairs is BC(t) by
    Definition 1, which ties the pair oracle to the Brandes oracle."""
    G = nx.gnp_random_graph(40, 0.08, seed=seed)
    e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
    g = gg.from_edges(40, e[:, 0], e[:, 1])
    acc = np.zeros(g.n)
    for u in range(g.n):
        dist, _, _ = O.brandes(g, u)
        for v in range(g.n):
            if u == v:
                continue
            y = O.pair_dependency(g, u, v)
            acc += y
            if dist[v] > 0:
                assert abs(y.sum() - (dist[v] - 1)) <= 1e-12 * max(1, dist[v])
            else:
                assert np.all(y == 0)
    bc = O.bc_exact(g)
    assert np.allclose(acc, bc, rtol=1e-11, atol=1e-9)


def test_pair_dependency_on_grid_beyond_fp64():
    g = gg.grid(600, 600)
    u, v = 0, 600 * 600 - 1
    y = O.pair_dependency(g, u, v)
    # on a full grid every vertex lies on some corner-to-corner shortest path
    assert np.all(np.isfinite(y))
    assert abs(y.sum() - (2 * 599 - 1)) <= 1e-9 * 2 * 599
    # the vertex next to the corner carries exactly half of the paths
    assert abs(y[1] - 0.5) < 1e-15 and abs(y[600] - 0.5) < 1e-15


# ------------------------------------------------------------ source sampler

def stream_sources(seed, k, n):
    return [(numpy_block(seed, 0, j)[0] * n) >> 64 for j in range(k)]


def stream_pairs(seed, k, n):
    out = []
    for j in range(k):
        w = numpy_block(seed, 1, j)
        u = (w[0] * n) >> 64
        v = (w[1] * (n - 1)) >> 64
        out.append((u, v + (v >= u)))
    return out


@pytest.mark.parametrize("n,c,seed", [(10, 1.0, 1), (10, 3.0, 2), (25, 2.5, 3), (7, 1.0, 9)])
def test_source_sampler_star_closed_form(n, c, seed):
    """Star centre: a leaf source contributes n-2, the centre itself 0
    (Definition 2), so S and the stopping k follow from the draws."""
    g = gg.star(n)
    draws = stream_sources(seed, 4000, n)
    S, k = 0, 0
    for s in draws:
        S += 0 if s == 0 else n - 2
        k += 1
        if S > c * n:
            break
    est, kk, SS, st = O.adaptive_source(g, [0], c, seed, k_max=10 ** 6)
    assert (kk[0], SS[0], st[0]) == (k, S, oracle.DONE)
    assert est[0] == (n * S) / k


@pytest.mark.parametrize("seed", range(1, 9))
def test_source_sampler_threshold_tie_path5(seed):
    """Path 0-1-2-3-4, target 2, c = 2: every sample adds 0 or 2 and c*n = 10
    is reachable exactly; the loop repeats while S <= c*n, so S = 10 does not
    stop it and it ends at S = 12."""
    g = gg.path(5)
    S, k = 0, 0
    for s in stream_sources(seed, 4000, 5):
        S += 0 if s == 2 else 2
        k += 1
        if S > 10:
            break
    assert S == 12
    est, kk, SS, st = O.adaptive_source(g, [2], 2.0, seed, k_max=10 ** 6)
    assert (kk[0], SS[0], st[0]) == (k, 12, oracle.DONE)
    assert est[0] == 5 * 12 / k


def test_source_sampler_capped_on_zero_bc_target():
    g = gg.star(12)
    est, k, S, st = O.adaptive_source(g, [3], 1.0, 5, k_max=37)
    assert (k[0], S[0], st[0], est[0]) == (37, 0.0, oracle.CAPPED, 0.0)


def test_source_sampler_targets_share_the_stream():
    g = gg.er(300, 0.03, seed=4)
    targets = gg.top_degree(g, 6)
    est, k, S, st = O.adaptive_source(g, targets, 2.0, 11, k_max=300)
    for i, t in enumerate(targets):
        e1, k1, S1, st1 = O.adaptive_source(g, [t], 2.0, 11, k_max=300)
        assert (est[i], k[i], S[i], st[i]) == (e1[0], k1[0], S1[0], st1[0])


def test_source_sampler_replays_dependencies():
    """The adaptive loop adds, in draw order, exactly the dependencies a plain
    Brandes pass gives for each drawn source."""
    g = gg.er(200, 0.04, seed=8)
    t = int(gg.top_degree(g, 1)[0])
    est, k, S, st = O.adaptive_source(g, [t], 3.0, 21, k_max=10 ** 6)
    draws = stream_sources(21, int(k[0]), g.n)
    full, _ = O.dependencies(g, np.array(draws, dtype=np.int32), full=True, total=False)
    acc = 0.0
    for i, s in enumerate(draws):
        acc += full[i][t]
        assert (acc > 3.0 * g.n) == (i == k[0] - 1)
    assert acc == S[0]


def test_source_sampler_unbiased_at_fixed_k():
    """With c too large to stop, the run ends at k_max and n*S/k is the mean of
    k i.i.d. draws of n*delta_s(v), whose expectation is BC(v) exactly when s
    is uniform over all n vertices (the target included)."""
    g = gg.from_edges(30, *np.array(list(nx.gnm_random_graph(30, 45, seed=2).edges())).T)
    bc = O.bc_exact(g)
    t = int(np.argmax(bc))
    kmax = 50
    ests = np.array([O.adaptive_source(g, [t], 1e9, seed, kmax)[0][0] for seed in range(2000)])
    se = ests.std(ddof=1) / np.sqrt(ests.shape[0])
    assert abs(ests.mean() - bc[t]) < 4 * se
    assert se < 0.01 * bc[t]


# -------------------------------------------------------------- pair sampler

@pytest.mark.parametrize("n,c,seed", [(8, 1.0, 1), (12, 2.0, 5)])
def test_pair_sampler_alg1_star(n, c, seed):
    """Star centre: a leaf-to-leaf pair passes the centre on its only shortest
    path (Y = 1), every pair with the centre as an end gives Y = 0."""
    g = gg.star(n)
    S, k = 0, 0
    for u, v in stream_pairs(seed, 100000, n):
        S += 1 if (u != 0 and v != 0) else 0
        k += 1
        if S > c * n:
            break
    est, kk, SS, st = O.adaptive_pair(g, [0], oracle.RULE_ALG1, 0.1, c, seed, 10 ** 7)
    assert (kk[0], SS[0], st[0]) == (k, S, oracle.DONE)
    assert est[0] == (n * (n - 1)) * S / k


@pytest.mark.parametrize("n,eps,seed", [(9, 0.1, 3), (30, 0.2, 4), (15, 0.45, 8)])
def test_pair_sampler_eps_rule_star(n, eps, seed):
    """Stop at the first k with S > 0 and k*S^2 >= eps^3 n^2."""
    g = gg.star(n)
    S, k = 0, 0
    rhs = eps ** 3 * n * n
    for u, v in stream_pairs(seed, 100000, n):
        S += 1 if (u != 0 and v != 0) else 0
        k += 1
        if S > 0 and k * S * S >= rhs:
            break
    est, kk, SS, st = O.adaptive_pair(g, [0], oracle.RULE_EPS, eps, 1.0, seed, 10 ** 7)
    assert (kk[0], SS[0], st[0]) == (k, S, oracle.DONE)


def test_pair_sampler_capped_and_shared():
    g = gg.path(9)
    est, k, S, st = O.adaptive_pair(g, [0, 4, 8], oracle.RULE_ALG1, 0.1, 1.0, 2, 500)
    assert st[0] == oracle.CAPPED and S[0] == 0 and k[0] == 500
    for i, t in enumerate([0, 4, 8]):
        e1, k1, S1, s1 = O.adaptive_pair(g, [t], oracle.RULE_ALG1, 0.1, 1.0, 2, 500)
        assert (est[i], k[i], S[i], st[i]) == (e1[0], k1[0], S1[0], s1[0])


def test_pair_sampler_unbiased_at_fixed_k():
    """n(n-1)*mean(Y) over uniform ordered pairs of distinct vertices has
    expectation BC(t) (the pair-sampling analogue of the source case)."""
    g = gg.from_edges(24, *np.array(list(nx.gnm_random_graph(24, 34, seed=6).edges())).T)
    bc = O.bc_exact(g)
    t = int(np.argmax(bc))
    kmax = 200
    ests = np.array([O.adaptive_pair(g, [t], oracle.RULE_ALG1, 0.1, 1e9, s, kmax)[0][0]
                     for s in range(1500)])
    se = ests.std(ddof=1) / np.sqrt(ests.shape[0])
    assert abs(ests.mean() - bc[t]) < 4 * se
    assert se < 0.012 * bc[t]


def test_sampler_argument_checks():
    g = gg.path(6)
    with pytest.raises(ValueError):
        O.adaptive_source(g, [1], 0.99, 1, 10)
    with pytest.raises(ValueError):
        O.adaptive_source(g, [6], 2.0, 1, 10)
    with pytest.raises(ValueError):
        O.adaptive_source(g, [1], 2.0, 1, 0)
    with pytest.raises(ValueError):
        O.adaptive_pair(g, [1], oracle.RULE_EPS, 0.5, 1.0, 1, 10)
    with pytest.raises(ValueError):
        O.adaptive_pair(g, [1], oracle.RULE_EPS, 0.0, 1.0, 1, 10)
    with pytest.raises(ValueError):
        O.adaptive_pair(g, [1], oracle.RULE_ALG1, 0.1, 0.5, 1, 10)
