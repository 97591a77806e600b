"""The profiler's work-unit counters against the oracle's work counts.

The roofline figure's numerator is (bytes per unit) x (units the kernels
count). These cases check the units themselves: over a source list, the
kernels must count exactly the (vertex, source) pairs and shortest-path DAG
edges that the oracle's plain BFS counts (oracle_source_work):
  discovery (top-down + bottom-up) units_a = sum over sources of (reached - 1)
  sigma_pull units_a = sum of (reached - 1);  units_b = sum of DAG edges
  backward units_a = sum of (reached - 1);
           units_b = sum of (DAG edges - deg(s)), the source's own edges being
           the only DAG edges the sweep from level 1 up does not read.
The two-sided pair search counts (bidir_pair) the vertices it adds (units_a)
and the arcs of every row it reads (units_b); both must equal the oracle's
count of the same walks (oracle_bidir_work) summed over the pairs.
Rows longer than 256 are summed in parts by their own kernel (hub_parts), whose
units_b hold those rows' DAG edges for both pulls: the two pulls' units_b and
hub_parts' add up to the two totals, and each pull alone matches its total on
a graph without such rows.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402

O = oracle.load()


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def expected(g, src):
    deg = g.degree()
    reach = dag = own = 0
    for s in src:
        r, _, d = O.source_work(g, int(s))
        reach += r - 1
        dag += d
        own += int(deg[s])
    return reach, dag, dag - own


def counted(G, src, dev, mode):
    G.profile(True)
    bc.dependencies(G, torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev), mode)
    prof = {k["name"]: k for k in G.profile_read()}
    G.profile(False)
    # the pair engine's persistent loops count discovery and path counts
    # together (pair_forward) and the sweep as pair_backward
    fwd = prof["pair_forward"]
    disc = prof["discover_topdown"]["units_a"] + prof["discover_bottomup"]["units_a"] + \
        fwd["units_a"]
    sa = prof["sigma_pull"]["units_a"] + fwd["units_a"]
    sb = prof["sigma_pull"]["units_b"] + fwd["units_b"]
    bwd_a = sum(prof[k]["units_a"] for k in ("backward", "pair_backward"))
    bwd_b = sum(prof[k]["units_b"] for k in ("backward", "pair_backward"))
    return disc, sa, sb, bwd_a, bwd_b, prof["hub_parts"]["units_b"]


CASES = [
    ("er2000 wave", lambda: gg.config_graph("er2000"), bc.BC_SCHED_BATCHED, 128, 0.0, 300),
    ("rmat12 pair engine per level", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9),
     -bc.BC_SCHED_THREADED, 128, 0.0, 300),
    ("er2000 wave bottom-up", lambda: gg.config_graph("er2000"), bc.BC_SCHED_BATCHED, 256, 1e-9,
     300),
    ("rmat12 wave", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9), bc.BC_SCHED_BATCHED, 512,
     0.0, 700),
    ("rmat12 pair engine level loop", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9),
     bc.BC_SCHED_THREADED, 128, 0.0, 300),
    ("grid60 pair engine level loop", lambda: gg.grid(60, 60), bc.BC_SCHED_THREADED, 64, 0.0,
     100),
]


@pytest.mark.parametrize("name,make,sched,batch,bu,k", CASES, ids=[c[0] for c in CASES])
def test_work_units_equal_the_oracle_counts(dev, name, make, sched, batch, bu, k):
    g = make()
    src = gg.philox_sources(5, k, g.n)
    src[:3] = gg.top_degree(g, 3)            # hubs, and a repeat of one
    src[7] = src[0]
    iso = np.flatnonzero(g.degree() == 0)
    if iso.size:
        src[9] = iso[0]                      # an isolated source reaches only itself
    reach, dag, bwd_dag = expected(g, src)
    G = bc.Graph(g.row, g.col)
    # a negative schedule id: that engine with one launch per level phase;
    # else the pair engine runs its persistent level loops
    G.configure(abs(sched), batch, bu, 0, -1 if sched < 0 else 1)
    sched = abs(sched)
    for mode in (bc.BC_OUT_SUM, bc.BC_OUT_FULL):
        say(name, "mode", mode)
        disc, sa, sb, ba, bb, hb = counted(G, src, dev, mode)
        assert G.stats()["schedule"] == sched
        assert disc == reach, (name, disc, reach)
        assert sa == reach, (name, sa, reach)
        assert ba == reach, (name, ba, reach)
        assert sb + bb + hb == dag + bwd_dag, (name, sb, bb, hb, dag, bwd_dag)
        if (g.degree() > 256).sum() == 0 or sched == bc.BC_SCHED_THREADED:
            assert hb == 0, (name, hb)
            assert sb == dag, (name, sb, dag)
            assert bb == bwd_dag, (name, bb, bwd_dag)
        else:
            assert hb > 0, name
    G.close()


@pytest.mark.parametrize("name,make", [("er2000", lambda: gg.config_graph("er2000")),
                                       ("grid60", lambda: gg.grid(60, 60)),
                                       ("rmat12", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19,
                                                                  seed=9))],
                         ids=["er2000", "grid60", "rmat12"])
def test_workgroup_units_equal_the_oracle_counts(dev, name, make):
    """One workgroup per source counts, per pass, every vertex it reaches
    besides the source (units_a) and every arc it walks (units_b): the rows of
    all reached vertices while discovering, and the in- and out-rows of every
    reached vertex but the source for the counts and the dependencies. On an
    undirected graph that is 3 * (sum of reached degrees) - 2 * deg(s), and the
    reached degrees sum to twice the edges of the source's component."""
    g = make()
    src = gg.philox_sources(8, 300, g.n)
    src[:3] = gg.top_degree(g, 3)
    src[7] = src[0]
    iso = np.flatnonzero(g.degree() == 0)
    if iso.size:
        src[9] = iso[0]
    deg = g.degree()
    want_a = want_b = 0
    for s in src:
        r, edges, _ = O.source_work(g, int(s))
        want_a += r - 1
        want_b += 3 * 2 * edges - 2 * int(deg[s])
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_WORKGROUP, 64, 0.0)
    for mode in (bc.BC_OUT_SUM, bc.BC_OUT_FULL):
        say(name, "workgroup mode", mode)
        G.profile(True)
        bc.dependencies(G, torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev), mode)
        prof = {k["name"]: k for k in G.profile_read()}
        G.profile(False)
        assert G.stats()["schedule"] == bc.BC_SCHED_WORKGROUP
        assert prof["wg_pass"]["units_a"] == want_a, (name, prof["wg_pass"]["units_a"], want_a)
        assert prof["wg_pass"]["units_b"] == want_b, (name, prof["wg_pass"]["units_b"], want_b)
    G.close()


@pytest.mark.parametrize("name,make", [("rmat12", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19,
                                                                  seed=9)),
                                       ("grid60", lambda: gg.grid(60, 60))],
                         ids=["rmat12", "grid60"])
def test_weighted_units_equal_the_oracle_counts(dev, name, make):
    """The weighted engine's count and dependency rounds each take every
    reached lane but the source once (units_a) and read its in-row or out-row
    (units_b); positive weights leave reachability as in the plain graph, so
    on an undirected graph units_a = sum of (reached - 1) and units_b = 2 *
    (component edges) - deg(s) per source. The search's units depend on the
    order in which rounds meet the lanes and are not compared."""
    g = gg.with_weights(make(), 9, seed=3)
    src = gg.philox_sources(8, 300, g.n)
    src[:3] = gg.top_degree(g, 3)
    src[7] = src[0]
    deg = g.degree()
    want_a = want_b = 0
    for s in src:
        r, edges, _ = O.source_work(g, int(s))
        want_a += r - 1
        want_b += 2 * edges - int(deg[s])
    G = bc.Graph(g.row, g.col, weights=g.w)
    G.configure(bc.BC_SCHED_AUTO, 128, 0.0)
    say(name, "weighted counters")
    G.profile(True)
    bc.dependencies(G, torch.from_numpy(np.ascontiguousarray(src, np.int32)).to(dev), bc.BC_OUT_SUM)
    prof = {k["name"]: k for k in G.profile_read()}
    G.profile(False)
    for k in ("w_counts", "w_backward"):
        assert prof[k]["units_a"] == want_a, (name, k, prof[k]["units_a"], want_a)
        assert prof[k]["units_b"] == want_b, (name, k, prof[k]["units_b"], want_b)
    assert prof["w_search"]["units_a"] >= want_b   # every reached lane's out-row at least once
    G.close()


BIDIR_CASES = [
    ("er2000", lambda: gg.config_graph("er2000"), False),
    ("rmat12", lambda: gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9), False),
    ("grid60", lambda: gg.grid(60, 60), False),
    ("drmat11", lambda: gg.rmat_directed(11, 8, 0.57, 0.19, 0.19, seed=4), True),
]


@pytest.mark.parametrize("name,make,directed", BIDIR_CASES, ids=[c[0] for c in BIDIR_CASES])
def test_bidir_units_equal_the_oracle_counts(dev, name, make, directed):
    g = make()
    rng = np.random.default_rng(31)
    us = rng.integers(0, g.n, 300).astype(np.int32)
    vs = rng.integers(0, g.n, 300).astype(np.int32)
    vs = np.where(vs == us, (vs + 1) % g.n, vs).astype(np.int32)
    top = gg.top_degree(g, 2)
    us[:2], vs[:2] = top, top[::-1]                       # hub to hub, both ways
    us[2], vs[2] = top[0], int(g.col[g.row[top[0]]])       # an arc's two ends
    iso = np.flatnonzero(g.degree() == 0)
    if iso.size:
        us[3], vs[3] = iso[0], top[0]                      # nothing to walk from u
        us[4], vs[4] = top[0], iso[0]
    want_a = want_b = 0
    for u, v in zip(us, vs):
        a, b = O.bidir_work(g, int(u), int(v), directed=directed)
        want_a += a
        want_b += b
    G = bc.Graph(g.row, g.col, directed=directed)
    G.configure(bc.BC_SCHED_AUTO, 0, 0.0, pair_search=bc.BC_PAIR_SEARCH_BIDIRECTIONAL)
    say(name, "two-sided search counters")
    G.profile(True)
    bc.pair_dependencies(G, torch.from_numpy(us).to(dev), torch.from_numpy(vs).to(dev))
    prof = {k["name"]: k for k in G.profile_read()}
    G.profile(False)
    assert G.stats()["pair_search"] == bc.BC_PAIR_SEARCH_BIDIRECTIONAL
    assert prof["bidir_pair"]["units_a"] == want_a, (name, prof["bidir_pair"]["units_a"], want_a)
    assert prof["bidir_pair"]["units_b"] == want_b, (name, prof["bidir_pair"]["units_b"], want_b)
    G.close()
