"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bars: distances bit-exact; path counts bit-exact below 2^53 and within 1e-12
relative above (extended values compared as m * 2^e); dependencies, BC, pair
dependencies and estimates within 1e-9 relative (values below 1e-290 in
magnitude on both sides count as equal); sample counts and statuses exact.
Every case prints its name before touching the GPU.
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
RTOL = 1e-9
TINY = 1e-290


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


def assert_close(got, want, rtol=RTOL, what=""):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, what
    tiny = (np.abs(got) < TINY) & (np.abs(want) < TINY)
    ok = tiny | (np.abs(got - want) <= rtol * np.abs(want))
    if not ok.all():
        i = np.flatnonzero(~ok.ravel())[:5]
        raise AssertionError("%s: %d mismatches, e.g. idx %s got %s want %s" % (
            what, int((~ok).sum()), i, got.ravel()[i], want.ravel()[i]))


def assert_sigma(gm, ge, om, oe, what=""):
    """Extended counts: identical below 2^53, 1e-12 relative above."""
    gm, ge, om, oe = (np.asarray(x) for x in (gm, ge, om, oe))
    small = (oe < 53) | (om == 0)
    assert np.array_equal(gm[small], om[small]) and np.array_equal(ge[small], oe[small]), what
    big = ~small
    if big.any():
        d = ge[big].astype(np.int64) - oe[big].astype(np.int64)
        assert np.all(np.abs(d) <= 1), what
        rel = np.abs(np.ldexp(gm[big], d) - om[big]) / om[big]
        assert rel.max() <= 1e-12, (what, rel.max())


def check_sources(G, g, src, dev, what):
    say(what, "n=%d k=%d" % (g.n, len(src)))
    full, dist, sig = bc.dependencies(G, T(src.astype(np.int32), dev), bc.BC_OUT_FULL,
                                      dist=True, sigma=True)
    full, dist = full.cpu().numpy(), dist.cpu().numpy()
    sm, se = sig[0].cpu().numpy(), sig[1].cpu().numpy()
    for i, s in enumerate(src):
        d, (om, oe), de = O.brandes(g, int(s))
        assert np.array_equal(dist[i], d), (what, "dist", i)
        assert_sigma(sm[i], se[i], om, oe, "%s sigma %d" % (what, i))
        assert_close(full[i], de, what="%s delta %d" % (what, i))
    return full


# ------------------------------------------------------------------ draws

@pytest.mark.parametrize("n", [2, 3, 2000, 1 << 20, 4194274])
def test_draws_bit_exact(dev, n):
    say("draws", n)
    g = gg.path(n)                       # draws depend only on n
    G = bc.Graph(g.row, g.col)
    for seed, j0, cnt in ((1, 0, 1000), (7, 123456789, 777), ((1 << 64) - 1, 5, 64)):
        u = torch.empty(cnt, dtype=torch.int32, device=dev)
        v = torch.empty(cnt, dtype=torch.int32, device=dev)
        bc.bc_draw_sources(G, seed, j0, cnt, u)
        want = [O.draw_source(seed, j0 + i, n) for i in range(cnt)]
        assert u.cpu().tolist() == want
        bc.bc_draw_pairs(G, seed, j0, cnt, u, v)
        want = [O.draw_pair(seed, j0 + i, n) for i in range(cnt)]
        assert list(zip(u.cpu().tolist(), v.cpu().tolist())) == want
    G.close()


def test_draws_bit_exact_large_n(dev):
    say("draws large n")
    g = gg.ba(1 << 20, 5, seed=7)
    G = bc.Graph(g.row, g.col)
    u = torch.empty(4096, dtype=torch.int32, device=dev)
    v = torch.empty(4096, dtype=torch.int32, device=dev)
    bc.bc_draw_sources(G, 7, 0, 4096, u)
    assert u.cpu().numpy().tolist() == gg.philox_sources(7, 4096, g.n).tolist()
    bc.bc_draw_pairs(G, 7, 99, 1000, u[:1000], v[:1000])
    want = [O.draw_pair(7, 99 + i, g.n) for i in range(1000)]
    assert list(zip(u[:1000].cpu().tolist(), v[:1000].cpu().tolist())) == want
    G.close()


# --------------------------------------------------------- Brandes passes

SMALL = [
    ("path17", lambda: gg.path(17)),
    ("star40", lambda: gg.star(40)),
    ("cycle9", lambda: gg.cycle(9)),
    ("cycle12", lambda: gg.cycle(12)),
    ("K12", lambda: gg.complete(12)),
    ("K3,5", lambda: gg.complete_bipartite(3, 5)),
    ("grid7x9", lambda: gg.grid(7, 9)),
    ("single", lambda: gg.from_edges(1, [], [])),
    ("edge", lambda: gg.path(2)),
    ("split", lambda: gg.from_edges(9, [0, 1, 3, 5, 6], [1, 2, 4, 6, 7])),
]


SCHEDS = [bc.BC_SCHED_BATCHED, bc.BC_SCHED_THREADED]
# every engine of bc_dependencies: wave per word, thread per pair, workgroup
# per source
ENGINES = SCHEDS + [bc.BC_SCHED_WORKGROUP]
ENGINE_IDS = ["wave", "pair", "wg"]
# pair samples: the one-sided search on each engine, and the two-sided search
ONE, BIDIR = bc.BC_PAIR_SEARCH_ONE_SIDED, bc.BC_PAIR_SEARCH_BIDIRECTIONAL
PAIR_SEARCHES = [(bc.BC_SCHED_BATCHED, ONE), (bc.BC_SCHED_THREADED, ONE),
                 (bc.BC_SCHED_AUTO, BIDIR)]
PAIR_IDS = ["wave", "pair", "bidir"]


@pytest.mark.parametrize("sched", ENGINES, ids=ENGINE_IDS)
@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_small_graphs_all_sources(dev, name, make, sched):
    g = make()
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0)
    src = np.arange(g.n, dtype=np.int32)
    check_sources(G, g, src, dev, name + " sched %d" % sched)
    assert G.stats()["schedule"] == sched
    out = bc.exact(G).cpu().numpy()
    assert_close(out, O.bc_exact(g), what=name + " bc")
    G.close()


@pytest.mark.parametrize("batch", [64, 128, 256])
@pytest.mark.parametrize("bottom_up", [-1.0, 0.0, 1e-9])
def test_er2000_batches_and_directions(dev, batch, bottom_up):
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, batch, bottom_up)
    src = gg.philox_sources(1, 200, g.n)          # 200 = several batches + ragged tail
    src[5] = src[77] = src[199] = 3               # repeats in and across batches
    check_sources(G, g, src, dev, "er2000 B=%d bu=%g" % (batch, bottom_up))
    G.close()


@pytest.mark.parametrize("batch", [64, 128])
def test_er2000_threaded_batches(dev, batch):
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_THREADED, batch, 0.0)
    src = gg.philox_sources(2, 150, g.n)
    src[3] = src[140] = 11
    check_sources(G, g, src, dev, "er2000 threaded B=%d" % batch)
    G.close()


def test_rmat_threaded_sum(dev):
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_THREADED, 128, 0.0)
    src = np.concatenate([np.flatnonzero(g.degree() == 0)[:2],
                          gg.philox_sources(8, 200, g.n)]).astype(np.int32)
    say("rmat12 threaded sum")
    out, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    _, want = O.dependencies(g, src, full=False, total=True)
    assert_close(out.cpu().numpy(), want, what="rmat12 threaded sum")
    G.close()


def test_auto_engine_selection(dev):
    say("auto engine")
    g = gg.grid(300, 300)
    G = bc.Graph(g.row, g.col)
    src = np.array([0, 4500, 89999], dtype=np.int32)
    check_sources(G, g, src, dev, "grid300 auto")
    assert G.stats()["schedule"] == bc.BC_SCHED_THREADED
    G.close()
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    bc.dependencies(G, T(np.array([0, 1999], np.int32), dev), bc.BC_OUT_SUM)
    assert G.stats()["schedule"] == bc.BC_SCHED_BATCHED
    G.close()


def test_er2000_exact_bc(dev):
    say("er2000 exact")
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    out = bc.exact(G).cpu().numpy()
    assert_close(out, O.bc_exact(g), what="er2000 bc")
    st = G.stats()
    assert st["samples_executed"] == g.n
    G.close()


def test_sum_mode_matches_oracle(dev):
    say("rmat12 sum")
    g = gg.rmat(12, 8, 0.57, 0.19, 0.19, seed=5)
    G = bc.Graph(g.row, g.col)
    src = gg.philox_sources(3, 300, g.n)
    out, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    _, want = O.dependencies(g, src, full=False, total=True)
    assert_close(out.cpu().numpy(), want, what="rmat12 sum")
    G.close()


@pytest.mark.parametrize("bu", [0.0, 1e-9], ids=["auto", "bottom-up"])
@pytest.mark.parametrize("batch", [64, 512])
def test_rmat_isolated_vertices_and_hubs(dev, batch, bu):
    # isolated sources end their search at level 0; bottom-up levels look only
    # for the lanes still present in the current level (1e-9: every level
    # bottom-up), which must not change any value
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    assert (g.degree() == 0).any()
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, batch, bu)
    iso = np.flatnonzero(g.degree() == 0)[:3]
    hubs = gg.top_degree(g, 3)
    src = np.concatenate([iso, hubs, gg.philox_sources(2, 90, g.n)]).astype(np.int32)
    check_sources(G, g, src, dev, "rmat12 B=%d bu=%g" % (batch, bu))
    G.close()


def test_grid_counts_beyond_2_53(dev):
    g = gg.grid(40, 40)
    G = bc.Graph(g.row, g.col)
    check_sources(G, g, np.array([0, 1599, 820, 41], dtype=np.int32), dev, "grid40")
    assert G.stats()["extended"] == 0
    G.close()


@pytest.mark.parametrize("sched", ENGINES, ids=ENGINE_IDS)
def test_grid_counts_beyond_fp64_range(dev, sched):
    g = gg.grid(600, 600)
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0)
    check_sources(G, g, np.array([0, 359999, 180300], dtype=np.int32), dev, "grid600")
    assert G.stats()["extended"] == 1
    G.close()


@pytest.mark.parametrize("sched", ENGINES, ids=ENGINE_IDS)
def test_hub_rows_with_extended_counts(dev, sched):
    # A 600x600 grid plus one hub joined to the 15x20 block of vertices in the
    # far corner: from the near corner the hub sits ~1166 levels deep, where
    # path counts are far beyond FP64's range, and its row (300 neighbours) is
    # longer than 256, so the wave engine sums it in two parts (extended counts).
    x = y = 600
    ids = np.arange(x * y).reshape(x, y)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    hub = x * y
    block = ids[585:600, 580:600].ravel()
    g = gg.from_edges(x * y + 1, np.concatenate([s, np.full(block.size, hub)]),
                      np.concatenate([d, block]), "grid600+hub")
    assert g.degree()[hub] == 300
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0)
    check_sources(G, g, np.array([0, hub, 359999, 180300], dtype=np.int32), dev,
                  "grid600+hub")
    assert G.stats()["extended"] == 1
    G.close()


def test_per_source_schedule(dev):
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_PER_SOURCE, 0, 0.0)
    src = gg.philox_sources(4, 20, g.n)
    say("per-source full")
    full, dist, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True)
    want, _ = O.dependencies(g, src, full=True, total=False)
    assert_close(full.cpu().numpy(), want, what="per-source full")
    for i, s in enumerate(src):
        assert np.array_equal(dist[i].cpu().numpy(), O.brandes(g, int(s))[0])
    say("per-source sum")
    out, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    assert_close(out.cpu().numpy(), want.sum(0), what="per-source sum")
    G.close()


def test_bit_identical_reruns_and_batch_positions(dev):
    g = gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=1)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, 128, 0.0)
    src = gg.philox_sources(5, 128, g.n)
    say("determinism")
    a = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL)[0].cpu().numpy()
    b = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL)[0].cpu().numpy()
    assert np.array_equal(a, b)
    # the same source alone, and at the last position of a different batch
    alone = bc.dependencies(G, T(src[:1], dev), bc.BC_OUT_FULL)[0].cpu().numpy()
    assert np.array_equal(alone[0], a[0])
    mixed = np.concatenate([gg.philox_sources(6, 127, g.n), src[:1]]).astype(np.int32)
    m = bc.dependencies(G, T(mixed, dev), bc.BC_OUT_FULL)[0].cpu().numpy()
    assert np.array_equal(m[127], a[0])
    G.close()


def test_lane_order_maps_rows_back(dev):
    """Samples are sorted by a clustering key before batching (from 128 on):
    per-source rows, distances and path counts must come back in the caller's
    order, bit-identical whatever the order of the list; sums may differ only
    by summation order. Pair mode maps (u, v) rows the same way."""
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, 128, 0.0)
    src = gg.philox_sources(11, 300, g.n)
    say("lane order rmat12 k=300")
    f1, d1, s1 = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True, sigma=True)
    rev = np.ascontiguousarray(src[::-1])
    f2, d2, s2 = bc.dependencies(G, T(rev, dev), bc.BC_OUT_FULL, dist=True, sigma=True)
    assert torch.equal(f1, f2.flip(0)) and torch.equal(d1, d2.flip(0))
    assert torch.equal(s1[0], s2[0].flip(0)) and torch.equal(s1[1], s2[1].flip(0))
    for i in (0, 150, 299):
        dd, _, de = O.brandes(g, int(src[i]))
        assert np.array_equal(d1[i].cpu().numpy(), dd)
        assert_close(f1[i].cpu().numpy(), de, what="lane order row %d" % i)
    a, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    b, _, _ = bc.dependencies(G, T(rev, dev), bc.BC_OUT_SUM)
    assert_close(a.cpu().numpy(), b.cpu().numpy(), rtol=1e-12, what="sum in both orders")
    assert_close(a.cpu().numpy(), f1.sum(0).cpu().numpy(), rtol=1e-12, what="sum vs rows")
    us = torch.empty(200, dtype=torch.int32, device=dev)
    vs = torch.empty(200, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 5, 0, 200, us, vs)
    p1 = bc.pair_dependencies(G, us, vs)
    p2 = bc.pair_dependencies(G, us.flip(0).contiguous(), vs.flip(0).contiguous())
    assert torch.equal(p1, p2.flip(0))
    for i in (0, 199):
        assert_close(p1[i].cpu().numpy(), O.pair_dependency(g, int(us[i]), int(vs[i])),
                     what="lane order pair %d" % i)
    G.close()


def test_invalid_arguments(dev):
    g = gg.path(6)
    G = bc.Graph(g.row, g.col)
    say("invalid args")
    with pytest.raises(bc.BcError) as e:
        bc.dependencies(G, T(np.array([0, 6], np.int32), dev))
    assert e.value.status == bc.BC_E_INVALID
    with pytest.raises(bc.BcError):
        bc.adaptive_source(G, T(np.array([1], np.int32), dev), 0.5, 1, 10)
    with pytest.raises(bc.BcError):
        bc.adaptive_pair(G, T(np.array([1], np.int32), dev), bc.BC_PAIR_EPS, 0.5, 1.0, 1, 10)
    with pytest.raises(bc.BcError):
        bc.pair_dependencies(G, T(np.array([2], np.int32), dev), T(np.array([2], np.int32), dev))
    with pytest.raises(bc.BcError):
        G.configure(bc.BC_SCHED_BATCHED, 96, 0.0)
    # empty source list is valid
    out, _, _ = bc.dependencies(G, T(np.zeros(0, np.int32), dev), bc.BC_OUT_SUM)
    assert np.all(out.cpu().numpy() == 0)
    G.close()


# --------------------------------------------------------- pair dependencies

@pytest.mark.parametrize("sched,search", PAIR_SEARCHES, ids=PAIR_IDS)
def test_pair_dependencies(dev, sched, search):
    g = gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=4)
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0, pair_search=search)
    r = np.random.default_rng(0)
    us = r.integers(0, g.n, 150).astype(np.int32)
    vs = r.integers(0, g.n - 1, 150).astype(np.int32)
    vs = vs + (vs >= us)
    nb = g.col[g.row[us[0]]:g.row[us[0] + 1]]
    if nb.shape[0]:
        vs[0] = nb[0]                                   # adjacent pair: no interior vertex
    iso = np.flatnonzero(g.degree() == 0)
    if iso.shape[0]:
        vs[1] = iso[0] if iso[0] != us[1] else iso[-1]  # unreachable destination
    say("pair deps", search)
    got = bc.pair_dependencies(G, T(us, dev), T(vs.astype(np.int32), dev)).cpu().numpy()
    assert G.stats()["pair_search"] == search
    for i in range(us.shape[0]):
        assert_close(got[i], O.pair_dependency(g, int(us[i]), int(vs[i])), what="pair %d" % i)
    G.close()


@pytest.mark.parametrize("search", [ONE, BIDIR], ids=["one", "bidir"])
@pytest.mark.parametrize("sched", ENGINES, ids=ENGINE_IDS)
def test_pair_dependencies_grid_extended(dev, sched, search):
    # corner to corner of the 600 x 600 grid: counts beyond 2^1000, so the
    # two-sided search hands the pairs to the one-sided engine
    g = gg.grid(600, 600)
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0, pair_search=search)
    us = np.array([0, 1000, 5], dtype=np.int32)
    vs = np.array([359999, 300000, 359000], dtype=np.int32)
    say("pair deps grid600", search)
    got = bc.pair_dependencies(G, T(us, dev), T(vs, dev)).cpu().numpy()
    assert G.stats()["pair_search"] == ONE
    for i in range(3):
        assert_close(got[i], O.pair_dependency(g, int(us[i]), int(vs[i])), what="gpair %d" % i)
    G.close()


def test_bidir_pairs_below_the_fp64_range(dev):
    # the 60 x 60 grid's corner-to-corner counts (C(118, 59) < 2^1000) stay
    # in the two-sided search; hubs, leaves, adjacent and unreachable pairs
    g = gg.grid(60, 60)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_AUTO, 0, 0.0, pair_search=BIDIR)
    us = np.array([0, 59, 1830, 0, 3599, 7], dtype=np.int32)
    vs = np.array([3599, 3540, 1769, 1, 0, 3000], dtype=np.int32)
    say("bidir grid60")
    got = bc.pair_dependencies(G, T(us, dev), T(vs, dev)).cpu().numpy()
    assert G.stats()["pair_search"] == BIDIR
    for i in range(us.shape[0]):
        assert_close(got[i], O.pair_dependency(g, int(us[i]), int(vs[i])), what="g60 %d" % i)
    h = gg.config_graph("er2000")
    H = bc.Graph(h.row, h.col)
    H.configure(bc.BC_SCHED_AUTO, 0, 0.0, pair_search=BIDIR)
    iso = np.flatnonzero(h.degree() == 0)
    hub = gg.top_degree(h, 2)
    us = np.array([hub[0], hub[1], iso[0] if iso.size else 3, 17], dtype=np.int32)
    vs = np.array([hub[1], 5, 9, iso[-1] if iso.size else 4], dtype=np.int32)
    vs = np.where(us == vs, (vs + 1) % h.n, vs).astype(np.int32)
    # more pairs than slots: each workgroup serves several in a row
    r = np.random.default_rng(8)
    ru = r.integers(0, h.n, 5000).astype(np.int32)
    rv = r.integers(0, h.n - 1, 5000).astype(np.int32)
    rv = rv + (rv >= ru)
    us, vs = np.concatenate([us, ru]), np.concatenate([vs, rv]).astype(np.int32)
    say("bidir er2000 5004 pairs")
    got = bc.pair_dependencies(H, T(us, dev), T(vs, dev)).cpu().numpy()
    assert H.stats()["pair_search"] == BIDIR
    for i in list(range(4)) + list(range(4, us.shape[0], 97)):
        assert_close(got[i], O.pair_dependency(h, int(us[i]), int(vs[i])), what="er %d" % i)
    # the same pairs again: slots reuse their state under new epochs
    again = bc.pair_dependencies(H, T(us, dev), T(vs, dev)).cpu().numpy()
    assert np.array_equal(got, again)
    G.close()
    H.close()


# --------------------------------------------------------------- samplers

def check_sampler(got, want, what):
    est, k, S, st = (x.cpu().numpy() for x in got)
    oest, ok, oS, ost = want
    assert np.array_equal(k, ok), (what, k, ok)
    assert np.array_equal(st, ost), what
    assert_close(S, oS, what=what + " S")
    assert_close(est, oest, what=what + " est")


@pytest.mark.parametrize("sched", SCHEDS, ids=["wave", "pair"])
def test_adaptive_source_er2000(dev, sched):
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0)
    targets = gg.top_degree(g, 16)
    say("adaptive source er2000")
    got = bc.adaptive_source(G, T(targets, dev), 5.0, 1, g.n)
    check_sampler(got, O.adaptive_source(g, targets, 5.0, 1, g.n), "source er2000")
    G.close()


@pytest.mark.parametrize("batch", [64, 256])
def test_adaptive_source_capped_and_shared(dev, batch):
    g = gg.rmat(10, 8, 0.57, 0.19, 0.19, seed=3)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, batch, 0.0)
    deg = g.degree()
    leaf = int(np.flatnonzero(deg == 1)[0])
    targets = np.array([leaf] + gg.top_degree(g, 5).tolist() + [leaf], dtype=np.int32)
    say("adaptive source capped B=%d" % batch)
    got = bc.adaptive_source(G, T(targets, dev), 1.5, 9, 300)
    want = O.adaptive_source(g, targets, 1.5, 9, 300)
    check_sampler(got, want, "source capped")
    assert want[3][0] == oracle.CAPPED
    G.close()


def test_adaptive_source_threshold_tie(dev):
    g = gg.path(5)
    G = bc.Graph(g.row, g.col)
    for seed in range(1, 6):
        say("tie seed", seed)
        got = bc.adaptive_source(G, T(np.array([2], np.int32), dev), 2.0, seed, 10 ** 6)
        check_sampler(got, O.adaptive_source(g, [2], 2.0, seed, 10 ** 6), "tie")
        assert got[2].cpu().numpy()[0] == 12.0
    G.close()


@pytest.mark.parametrize("sched,search", PAIR_SEARCHES, ids=PAIR_IDS)
def test_adaptive_pair_eps_er2000(dev, sched, search):
    g = gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0, pair_search=search)
    targets = gg.top_degree(g, 16)
    say("adaptive pair eps er2000", search)
    got = bc.adaptive_pair(G, T(targets, dev), bc.BC_PAIR_EPS, 0.1, 1.0, 1, 1 << 20)
    check_sampler(got, O.adaptive_pair(g, targets, oracle.RULE_EPS, 0.1, 1.0, 1, 1 << 20),
                  "pair eps er2000")
    assert G.stats()["pair_search"] == search
    G.close()


@pytest.mark.parametrize("sched,search", PAIR_SEARCHES, ids=PAIR_IDS)
def test_adaptive_pair_alg1_small(dev, sched, search):
    g = gg.er(150, 0.04, seed=2)
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0, pair_search=search)
    targets = gg.top_degree(g, 3)
    say("adaptive pair alg1", search)
    got = bc.adaptive_pair(G, T(targets, dev), bc.BC_PAIR_ALG1, 0.1, 1.0, 5, 1 << 20)
    check_sampler(got, O.adaptive_pair(g, targets, oracle.RULE_ALG1, 0.1, 1.0, 5, 1 << 20),
                  "pair alg1")
    G.close()


def test_accuracy_sweep_settings_match_the_oracle(dev):
    # the sweep's settings run through the library's samplers: the same
    # streams give the oracle's sample counts and estimates
    import paper_1608_04472_amd.accuracy as acc
    g = gg.powerlaw_cluster(700, 2, 0.4, seed=5)
    G = bc.Graph(g.row, g.col)
    exact = bc.exact(G).cpu().numpy()
    _, want_bc = O.dependencies(g, np.arange(g.n, dtype=np.int32), full=False, total=True)
    assert_close(exact, want_bc, what="sweep exact")
    tg = acc.top_targets(exact, 6)
    say("accuracy sweep settings")
    for kind, prm in (("source", 1.5), ("pair-eps", 0.2), ("pair-alg1", 1.0)):
        K, D, capped, _ = acc.run_setting(bc, G, T(tg, dev), exact[tg], kind, prm, 2, 1 << 20)
        for inst in range(2):
            if kind == "source":
                est, k, _, _ = O.adaptive_source(g, tg, prm, 1 + inst, 1 << 20)
            elif kind == "pair-eps":
                est, k, _, _ = O.adaptive_pair(g, tg, oracle.RULE_EPS, prm, 1.0, 1 + inst, 1 << 20)
            else:
                est, k, _, _ = O.adaptive_pair(g, tg, oracle.RULE_ALG1, 0.1, prm, 1 + inst,
                                               1 << 20)
            assert np.array_equal(K[inst], k), (kind, inst)
            assert_close(D[inst], np.abs(est / want_bc[tg] - 1.0), what=kind)
        assert capped == 0
    G.close()


@pytest.mark.parametrize("bu", [0.0, 1e-9], ids=["auto", "bottom-up"])
def test_long_rows_in_parts_bit_identical_across_widths(dev, bu):
    # rows longer than 256 are summed in fixed parts of 256 (each by its own
    # wavefront, parts added in order) and shorter rows in CSR order, so a
    # source's values do not depend on the batch it runs in: widths 64, 512
    # and 4096 (one, eight and 64 words of 64) give identical bits, and they
    # match the oracle; with every level bottom-up, those rows also look for
    # their frontier parents with a wavefront each
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    assert (g.degree() > 256).sum() > 20 and g.degree().max() > 4 * 256
    src = np.concatenate([gg.top_degree(g, 4), gg.philox_sources(4, 250, g.n)]).astype(np.int32)
    outs = {}
    for width in (64, 512, 4096):
        G = bc.Graph(g.row, g.col)
        G.configure(bc.BC_SCHED_BATCHED, width, bu)
        if width == 64:
            outs[width] = check_sources(G, g, src, dev, "rmat12 parts width 64 bu=%g" % bu)
        else:
            say("rmat12 parts width %d bu=%g" % (width, bu))
            outs[width] = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL)[0].cpu().numpy()
        assert G.stats()["batch_width"] == width
        G.close()
    assert np.array_equal(outs[64], outs[512])
    assert np.array_equal(outs[64], outs[4096])


@pytest.mark.parametrize("what", ["grid600 extended", "rmat12 pairs", "grid90 sampler"])
def test_pair_engine_level_loop_equals_per_level(dev, what):
    """The pair engine's persistent level loops (one launch per pass, grid
    barriers between phases) and its one-launch-per-phase form do the same
    additions in the same order: identical bits, and the oracle's values."""
    outs = []
    for loop in (1, -1):
        if what == "grid600 extended":
            g = gg.grid(600, 600)
            G = bc.Graph(g.row, g.col)
            G.configure(bc.BC_SCHED_THREADED, 64, 0.0, 0, loop)
            src = np.array([0, 359999, 180300, 7], dtype=np.int32)
            say("level loop", loop, what)
            full, dist, sig = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True,
                                              sigma=True)
            assert G.stats()["extended"] == 1
            outs.append([full.cpu().numpy(), dist.cpu().numpy(), sig[0].cpu().numpy(),
                         sig[1].cpu().numpy()])
            if loop == 1:
                for i in (0, 2):
                    d, (om, oe), de = O.brandes(g, int(src[i]))
                    assert np.array_equal(outs[-1][1][i], d)
                    assert_sigma(outs[-1][2][i], outs[-1][3][i], om, oe, "loop sigma")
                    assert_close(outs[-1][0][i], de, what="loop delta")
        elif what == "rmat12 pairs":
            g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
            G = bc.Graph(g.row, g.col)
            G.configure(bc.BC_SCHED_THREADED, 128, 0.0, 0, loop)
            us = torch.empty(300, dtype=torch.int32, device=dev)
            vs = torch.empty(300, dtype=torch.int32, device=dev)
            bc.bc_draw_pairs(G, 4, 0, 300, us, vs)
            say("level loop", loop, what)
            p = bc.pair_dependencies(G, us, vs).cpu().numpy()
            src = gg.philox_sources(9, 300, g.n)
            tot, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
            outs.append([p, tot.cpu().numpy()])
            if loop == 1:
                for i in (0, 299):
                    assert_close(p[i], O.pair_dependency(g, int(us[i]), int(vs[i])),
                                 what="loop pair %d" % i)
                _, want = O.dependencies(g, src, full=False, total=True)
                assert_close(outs[-1][1], want, what="loop sum")
        else:
            g = gg.grid(90, 90)
            G = bc.Graph(g.row, g.col)
            G.configure(bc.BC_SCHED_THREADED, 0, 0.0, 0, loop)
            tg = np.array([4095, 4050, 45], dtype=np.int32)
            say("level loop", loop, what)
            a = bc.adaptive_source(G, T(tg, dev), 2.0, 3, 500)
            b = bc.adaptive_pair(G, T(tg, dev), bc.BC_PAIR_EPS, 0.2, 1.0, 3, 3000)
            outs.append([x.cpu().numpy() for x in a + b])
            if loop == 1:
                check_sampler(a, O.adaptive_source(g, tg, 2.0, 3, 500), "loop source")
                check_sampler(b, O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.2, 1.0, 3, 3000),
                              "loop pair")
        G.close()
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y), what


def test_workgroup_engine_outputs_and_slots(dev):
    """Workgroup per source: BC_OUT_SUM (per-slot sums reduced in slot order),
    BC_OUT_TARGETS, one-sided pair rows, and more sources than slots (each
    workgroup runs several passes, resetting its distances in between)."""
    g = gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=4)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_WORKGROUP, 64, 0.0, pair_search=ONE)
    src = gg.philox_sources(9, 700, g.n)
    src[:3] = gg.top_degree(g, 3)
    src[5] = src[0]
    say("wg rmat11 700 sources on 64 slots")
    full, want = O.dependencies(g, src, full=True, total=True)
    tot, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    assert G.stats()["schedule"] == bc.BC_SCHED_WORKGROUP and G.stats()["batch_width"] == 64
    assert_close(tot.cpu().numpy(), want, what="wg sum")
    again, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    assert torch.equal(tot, again)
    tg = gg.top_degree(g, 6)
    got = bc.target_dependencies(G, T(src, dev), T(tg, dev)).cpu().numpy()
    assert_close(got, full[:, tg], what="wg targets")
    rows, _, _ = bc.dependencies(G, T(src[:150], dev), bc.BC_OUT_FULL)
    assert_close(rows.cpu().numpy(), full[:150], what="wg rows")
    us = torch.empty(120, dtype=torch.int32, device=dev)
    vs = torch.empty(120, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 4, 0, 120, us, vs)
    say("wg one-sided pairs")
    p = bc.pair_dependencies(G, us, vs).cpu().numpy()
    assert G.stats()["pair_search"] == ONE
    u, v = us.cpu().numpy(), vs.cpu().numpy()
    for i in range(0, 120, 5):
        assert_close(p[i], O.pair_dependency(g, int(u[i]), int(v[i])), what="wg pair %d" % i)
    G.close()
