"""Weighted graphs on the GPU (bc_graph_create_weighted) against the
weighted oracle (Dijkstra's algorithm, Section 3): distances bit-exact, path
counts exact below 2^53, dependencies, exact BC, pair dependencies and both
samplers within the tolerance of the other parity tests; undirected and
directed; batches of 64 to 4096 sources (one to 64 words of 64) with ragged
tails, rows longer than one search task; unit weights give
the unweighted library's values; counts beyond 2^1000 are refused."""
import sys
from dataclasses import replace

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402
from test_gpu_parity import assert_close, assert_sigma, check_sampler  # noqa: E402

O = oracle.load()


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def T(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(dev)


def wgraph(g):
    return bc.Graph(g.row, g.col, directed=g.directed, weights=g.w)


def check_sources(G, g, src, dev, what):
    say(what, "n=%d k=%d" % (g.n, len(src)))
    full, dist, sig = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True, sigma=True)
    full, dist = full.cpu().numpy(), dist.cpu().numpy()
    sm, se = sig[0].cpu().numpy(), sig[1].cpu().numpy()
    for i, s in enumerate(src):
        d, (om, oe), de = O.brandes(g, int(s), directed=g.directed)
        assert np.array_equal(dist[i], d), (what, "dist", i)
        assert_sigma(sm[i], se[i], om, oe, "%s sigma %d" % (what, i))
        assert_close(full[i], de, what="%s delta %d" % (what, i))


def small_cases():
    out = []
    for directed in (False, True):
        for seed in range(4):
            r = np.random.default_rng(40 + seed)
            n = int(r.integers(6, 30))
            m = int(r.integers(n, 4 * n))
            a, b = r.integers(0, n, m), r.integers(0, n, m)
            g = gg.from_arcs(n, a, b) if directed else gg.from_edges(n, a, b)
            out.append(("%s%d" % ("d" if directed else "u", seed), gg.with_weights(g, 3, seed)))
    return out


SMALL = small_cases()


@pytest.mark.parametrize("name,g", SMALL, ids=[c[0] for c in SMALL])
def test_small_weighted_all_sources(dev, name, g):
    G = wgraph(g)
    check_sources(G, g, np.arange(g.n, dtype=np.int32), dev, name)
    assert_close(bc.exact(G).cpu().numpy(), O.bc_exact(g, directed=g.directed),
                 what=name + " bc")
    assert G.stats()["schedule"] == bc.BC_SCHED_BATCHED
    G.close()


@pytest.mark.parametrize("directed", [False, True], ids=["undirected", "directed"])
@pytest.mark.parametrize("batch", [64, 512, 4096])
def test_rmat_weighted_batches(dev, directed, batch):
    base = gg.rmat_directed(11, 8, 0.57, 0.19, 0.19, seed=5) if directed else \
        gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=5)
    g = gg.with_weights(base, 10, seed=5)
    G = wgraph(g)
    G.configure(bc.BC_SCHED_AUTO, batch, 0.0)
    src = gg.philox_sources(3, 300, g.n)          # several batches, a ragged tail
    src[:3] = gg.top_degree(g, 3)
    src[7] = src[0]
    check_sources(G, g, src, dev, "wrmat11 B=%d" % batch)
    say("wrmat11 sum and targets")
    tot, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    full, want = O.dependencies(g, src, full=True, total=True, directed=directed)
    assert_close(tot.cpu().numpy(), want, what="wrmat11 sum")
    tg = gg.top_degree(g, 5)
    got = bc.target_dependencies(G, T(src, dev), T(tg, dev)).cpu().numpy()
    assert_close(got, full[:, tg], what="wrmat11 targets")
    G.close()


def test_weighted_pairs_and_samplers(dev):
    g = gg.with_weights(gg.rmat(10, 8, 0.57, 0.19, 0.19, seed=6), 6, seed=6)
    G = wgraph(g)
    r = np.random.default_rng(2)
    us = r.integers(0, g.n, 120).astype(np.int32)
    vs = r.integers(0, g.n - 1, 120).astype(np.int32)
    vs = vs + (vs >= us)
    nb = g.col[g.row[us[0]]:g.row[us[0] + 1]]
    if nb.shape[0]:
        vs[0] = nb[0]
    iso = np.flatnonzero(g.degree() == 0)
    if iso.shape[0]:
        vs[1] = iso[0] if iso[0] != us[1] else iso[-1]
    say("weighted pairs")
    got = bc.pair_dependencies(G, T(us, dev), T(vs.astype(np.int32), dev)).cpu().numpy()
    assert G.stats()["pair_search"] == bc.BC_PAIR_SEARCH_ONE_SIDED
    for i in range(us.shape[0]):
        assert_close(got[i], O.pair_dependency(g, int(us[i]), int(vs[i])), what="wpair %d" % i)
    tg = gg.top_degree(g, 4)
    say("weighted samplers")
    check_sampler(bc.adaptive_source(G, T(tg, dev), 2.0, 5, 1500),
                  O.adaptive_source(g, tg, 2.0, 5, 1500), "wsource")
    check_sampler(bc.adaptive_pair(G, T(tg, dev), bc.BC_PAIR_EPS, 0.2, 1.0, 5, 20000),
                  O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.2, 1.0, 5, 20000), "wpair eps")
    G.close()


def test_unit_weights_equal_the_unweighted_library(dev):
    g = gg.grid(40, 40)
    src = T(gg.philox_sources(4, 200, g.n), dev)
    U = bc.Graph(g.row, g.col)
    W = bc.Graph(g.row, g.col, weights=np.ones(g.nnz, np.int32))
    say("unit weights grid40")
    a, da, _ = bc.dependencies(U, src, bc.BC_OUT_FULL, dist=True)
    b, db, _ = bc.dependencies(W, src, bc.BC_OUT_FULL, dist=True)
    assert torch.equal(da, db)
    assert_close(b.cpu().numpy(), a.cpu().numpy(), what="unit weights")
    U.close()
    W.close()


def test_counts_beyond_fp64_are_refused(dev):
    # unit weights on the 600 x 600 grid: corner-to-corner counts pass 2^1000
    g = gg.grid(600, 600)
    G = bc.Graph(g.row, g.col, weights=np.ones(g.nnz, np.int32))
    say("weighted grid600 overflow")
    with pytest.raises(bc.BcError) as e:
        bc.dependencies(G, T(np.array([0], np.int32), dev), bc.BC_OUT_SUM)
    assert e.value.status == bc.BC_E_UNSUPPORTED
    # the graph stays usable for sources whose counts fit
    src = np.array([180300], np.int32)
    h = replace(g, w=np.ones(g.nnz, np.int32))
    full, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL)
    _, _, de = O.brandes(h, int(src[0]))
    assert_close(full.cpu().numpy()[0], de, what="grid600 centre")
    G.close()


def test_weighted_graph_rejections(dev):
    g = gg.with_weights(gg.path(6), 4, seed=1)
    G = wgraph(g)
    say("weighted rejections")
    with pytest.raises(bc.BcError) as e:
        out = torch.zeros(g.n, dtype=torch.float64, device=dev)
        bc.bc_dependencies_noalloc(G, T(np.array([0], np.int32), dev), bc.BC_OUT_SUM, out)
    assert e.value.status == bc.BC_E_UNSUPPORTED
    G.close()
    with pytest.raises(bc.BcError) as e:
        bc.Graph(g.row, g.col, weights=np.where(np.arange(g.nnz) == 1, 0, g.w))
    assert e.value.status == bc.BC_E_INVALID
    asym = g.w.copy()
    asym[0] += 1
    with pytest.raises(bc.BcError) as e:
        bc.Graph(g.row, g.col, weights=asym)
    assert e.value.status == bc.BC_E_INVALID
