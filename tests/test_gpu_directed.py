"""Directed graphs on the GPU (bc_graph_create_directed) against the oracle's
directed functions: distances bit-exact, path counts bit-exact below 2^53,
dependencies, BC, pair dependencies and estimates within 1e-9, sample counts
exact; a bidirected graph gives the undirected handle's bits.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402
from test_gpu_parity import (PAIR_IDS, PAIR_SEARCHES, assert_close, assert_sigma,  # noqa: E402
                             check_sampler)

O = oracle.load()
SCHEDS = [bc.BC_SCHED_BATCHED, bc.BC_SCHED_THREADED]


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def T(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def digraph(seed, n):
    r = np.random.default_rng(seed)
    m = 3 * n
    return gg.from_arcs(n, r.integers(0, n, m), r.integers(0, n, m), "dg%d" % seed)


def check_sources(G, g, src, dev, what):
    say(what, "n=%d k=%d" % (g.n, len(src)))
    full, dist, sig = bc.dependencies(G, T(src.astype(np.int32), dev), bc.BC_OUT_FULL,
                                      dist=True, sigma=True)
    full, dist = full.cpu().numpy(), dist.cpu().numpy()
    sm, se = sig[0].cpu().numpy(), sig[1].cpu().numpy()
    for i, s in enumerate(src):
        d, (om, oe), de = O.brandes(g, int(s), directed=True)
        assert np.array_equal(dist[i], d), (what, "dist", i)
        assert_sigma(sm[i], se[i], om, oe, "%s sigma %d" % (what, i))
        assert_close(full[i], de, what="%s delta %d" % (what, i))


SMALL = [("dpath12", lambda: gg.directed_path(12)), ("dcycle9", lambda: gg.directed_cycle(9)),
         ("ostar10", lambda: gg.out_star(10)), ("dg1", lambda: digraph(1, 40)),
         ("dg2", lambda: digraph(2, 300))]


@pytest.mark.parametrize("sched", SCHEDS + [bc.BC_SCHED_PER_SOURCE, bc.BC_SCHED_WORKGROUP],
                         ids=["wave", "pair", "per-source", "wg"])
@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_small_digraphs_all_sources(dev, name, make, sched):
    g = make()
    G = bc.Graph(g.row, g.col, directed=True)
    G.configure(sched, 0, 0.0)
    src = np.arange(g.n, dtype=np.int32)
    if sched == bc.BC_SCHED_PER_SOURCE:
        say(name, "per-source")
        full, dist, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True)
        want, _ = O.dependencies(g, src, full=True, total=False, directed=True)
        assert_close(full.cpu().numpy(), want, what=name + " per-source")
    else:
        check_sources(G, g, src, dev, name + " sched %d" % sched)
    assert_close(bc.exact(G).cpu().numpy(), O.bc_exact(g, directed=True), what=name + " bc")
    G.close()


@pytest.mark.parametrize("batch,bottom_up", [(64, -1.0), (256, 0.0), (512, 1e-9), (4096, 0.0)])
def test_rmat_directed_batches(dev, batch, bottom_up):
    g = gg.rmat_directed(12, 16, 0.57, 0.19, 0.19, seed=9)
    G = bc.Graph(g.row, g.col, directed=True)
    G.configure(bc.BC_SCHED_BATCHED, batch, bottom_up)
    src = gg.philox_sources(3, 300, g.n)
    src[:3] = gg.top_degree(g, 3)
    check_sources(G, g, src, dev, "drmat12 B=%d bu=%g" % (batch, bottom_up))
    say("drmat12 sum")
    tot, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    _, want = O.dependencies(g, src, full=False, total=True, directed=True)
    assert_close(tot.cpu().numpy(), want, what="drmat12 sum")
    G.close()


@pytest.mark.parametrize("sched,search", PAIR_SEARCHES, ids=PAIR_IDS)
def test_directed_pairs_and_samplers(dev, sched, search):
    g = gg.rmat_directed(11, 8, 0.57, 0.19, 0.19, seed=4)
    G = bc.Graph(g.row, g.col, directed=True)
    G.configure(sched, 0, 0.0, pair_search=search)
    us = torch.empty(200, dtype=torch.int32, device=dev)
    vs = torch.empty(200, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 3, 0, 200, us, vs)
    say("directed pairs", sched)
    got = bc.pair_dependencies(G, us, vs).cpu().numpy()
    u, v = us.cpu().numpy(), vs.cpu().numpy()
    for i in range(0, 200, 7):
        assert_close(got[i], O.pair_dependency(g, int(u[i]), int(v[i]), directed=True),
                     what="dpair %d" % i)
    tg = gg.top_degree(g, 4)
    say("directed samplers", sched)
    check_sampler(bc.adaptive_source(G, T(tg, dev), 2.0, 5, 1500),
                  O.adaptive_source(g, tg, 2.0, 5, 1500, directed=True), "dsource")
    check_sampler(bc.adaptive_pair(G, T(tg, dev), bc.BC_PAIR_EPS, 0.2, 1.0, 5, 20000),
                  O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.2, 1.0, 5, 20000, directed=True),
                  "dpair eps")
    G.close()


def test_bidirected_equals_undirected(dev):
    g = gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=6)
    src = T(gg.philox_sources(2, 200, g.n), dev)
    say("bidirected")
    U = bc.Graph(g.row, g.col)
    D = bc.Graph(g.row, g.col, directed=True)
    for sched in SCHEDS:
        U.configure(sched, 128, 0.0)
        D.configure(sched, 128, 0.0)
        a = bc.dependencies(U, src, bc.BC_OUT_FULL)[0]
        b = bc.dependencies(D, src, bc.BC_OUT_FULL)[0]
        assert torch.equal(a, b)
    U.close()
    D.close()


def test_directed_validation(dev):
    import ctypes
    lib = bc.load_library()
    h = ctypes.c_void_p()
    # an asymmetric CSR is a valid digraph; a self-loop is not
    row = np.array([0, 1, 1], dtype=np.int64)
    col = np.array([1], dtype=np.int32)
    csr = bc._Csr(2, 1, row.ctypes.data, 1, col.ctypes.data)
    assert lib.bc_graph_create_directed(ctypes.byref(csr), None, None, ctypes.byref(h)) == \
        bc.BC_OK
    lib.bc_graph_destroy(h)
    row = np.array([0, 1, 1], dtype=np.int64)
    col = np.array([0], dtype=np.int32)
    csr = bc._Csr(2, 1, row.ctypes.data, 1, col.ctypes.data)
    assert lib.bc_graph_create_directed(ctypes.byref(csr), None, None, ctypes.byref(h)) == \
        bc.BC_E_INVALID
