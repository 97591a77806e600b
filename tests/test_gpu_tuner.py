"""The autotuner: every plan it can pick gives the oracle's values, and what
it picks comes from its candidate set, is cached per graph signature, and
keeps results equal to the untuned library's.

Candidates (bc_graph_tune): the wave engine at widths 256 .. 4096 with
bottom_up in {0.04, 0.01, 0.15, never}, the pair engine at widths 256 .. 4096 with and without its
persistent level loop, and one workgroup per source with 64 .. 1024
sources in flight (on graphs deeper than 32 levels or of at most 2^16
vertices).
"""
import itertools
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402
from test_gpu_parity import assert_close  # noqa: E402

O = oracle.load()
WIDTHS = [256, 512, 1024, 2048, 4096]
WG_WIDTHS = [64, 128, 256, 512, 1024]
BOTTOM_UP = [0.04, 0.01, 0.15, -1.0]
WAVE_PLANS = list(itertools.product(WIDTHS, BOTTOM_UP))
PAIR_PLANS = list(itertools.product(WIDTHS, [-1, 1]))


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def case(dev):
    g = gg.rmat(11, 16, 0.57, 0.19, 0.19, seed=3)
    src = gg.philox_sources(13, 300, g.n)
    src[:2] = gg.top_degree(g, 2)
    full, tot = O.dependencies(g, src, full=True, total=True)
    G = bc.Graph(g.row, g.col)
    yield g, G, torch.from_numpy(src).to(dev), full, tot
    G.close()


def check(G, s, full, tot, what):
    out, _, _ = bc.dependencies(G, s, bc.BC_OUT_FULL)
    assert_close(out.cpu().numpy(), full, what=what + " rows")
    out, _, _ = bc.dependencies(G, s, bc.BC_OUT_SUM)
    assert_close(out.cpu().numpy(), tot, what=what + " sum")


def test_every_wave_plan(case):
    g, G, s, full, tot = case
    for B, bu in WAVE_PLANS:
        say("wave plan", B, bu)
        G.configure(bc.BC_SCHED_BATCHED, B, bu)
        check(G, s, full, tot, "wave B=%d bu=%g" % (B, bu))
        assert G.stats()["batch_width"] == B


def test_every_workgroup_plan(case):
    g, G, s, full, tot = case
    for B in WG_WIDTHS:
        say("workgroup plan", B)
        G.configure(bc.BC_SCHED_WORKGROUP, B, 0.0)
        check(G, s, full, tot, "wg B=%d" % B)
        assert G.stats()["batch_width"] == min(B, s.numel())


def test_every_pair_plan(case):
    g, G, s, full, tot = case
    for B, loop in PAIR_PLANS:
        say("pair plan", B, loop)
        G.configure(bc.BC_SCHED_THREADED, B, 0.0, 0, loop)
        check(G, s, full, tot, "pair B=%d loop=%d" % (B, loop))
        assert G.stats()["batch_width"] == B


@pytest.mark.parametrize("name", ["rmat12", "grid60"])
def test_tuned_plan(dev, name):
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9) if name == "rmat12" else gg.grid(60, 60)
    G = bc.Graph(g.row, g.col)
    say("tune", name)
    plan = G.tune()
    assert plan["schedule"] in (bc.BC_SCHED_BATCHED, bc.BC_SCHED_THREADED,
                                bc.BC_SCHED_WORKGROUP)
    assert plan["batch"] in WIDTHS + WG_WIDTHS
    if plan["schedule"] == bc.BC_SCHED_WORKGROUP:
        assert plan["batch"] in WG_WIDTHS
    elif plan["schedule"] == bc.BC_SCHED_BATCHED:
        assert plan["bottom_up"] in BOTTOM_UP + [0.0] and plan["split_entries"] == 0
    else:
        assert plan["level_loop"] in (0, 1, -1)
    eff = G.plan()
    assert eff["schedule"] == plan["schedule"] and eff["batch"] == plan["batch"]
    src = gg.philox_sources(17, 200, g.n)
    full, tot = O.dependencies(g, src, full=True, total=True)
    check(G, torch.from_numpy(src).to(dev), full, tot, "tuned " + name)
    # a second handle of the same graph finds the plan in the cache
    H = bc.Graph(g.row, g.col)
    H.configure(bc.BC_SCHED_TUNED)
    assert H.plan() == eff
    tg = gg.top_degree(g, 3)
    est = bc.adaptive_source(H, torch.from_numpy(tg).to(dev), 2.0, 5, 300)
    want = O.adaptive_source(g, tg, 2.0, 5, 300)
    assert np.array_equal(est[1].cpu().numpy(), want[1])
    assert_close(est[0].cpu().numpy(), want[0], what="tuned sampler")
    H.close()
    G.close()


@pytest.mark.parametrize("name", ["rmat12", "er2000"])
def test_sampler_rounds_take_a_threshold_tried_at_their_width(dev, name):
    """A source sampler whose round width differs from the tuned plan's runs
    the wave engine with a bottom-up threshold tried at the round width: one of
    the candidates, the same on a second call (kept per graph and width), the
    plan itself left as tuned, and the estimates equal to the oracle's."""
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9) if name == "rmat12" else \
        gg.config_graph("er2000")
    G = bc.Graph(g.row, g.col)
    say("tune", name)
    plan = G.tune()
    sb = 512 if plan["batch"] == 256 else 256
    H = bc.Graph(g.row, g.col)
    H.configure(bc.BC_SCHED_TUNED, 0, 0.0, 0, 0, sb)
    eff = H.plan()
    tg = gg.top_degree(g, 3)
    want = O.adaptive_source(g, tg, 2.0, 5, 300)
    used = []
    for rep in range(2):
        say("sampler rounds", name, "width", sb, "call", rep)
        est = bc.adaptive_source(H, torch.from_numpy(tg).to(dev), 2.0, 5, 300)
        assert np.array_equal(est[1].cpu().numpy(), want[1])
        assert_close(est[0].cpu().numpy(), want[0], what="sampler at width %d" % sb)
        st = H.stats()
        assert st["batch_width"] == sb
        used.append(st["bottom_up"])
        assert H.plan() == eff
    if eff["schedule"] == bc.BC_SCHED_BATCHED:
        assert used[0] in BOTTOM_UP, used
        assert used[1] == used[0], used
    else:
        assert used == [0.0, 0.0], used      # the wave engine did not run
    # the plan's own width keeps the plan's threshold
    H.configure(bc.BC_SCHED_TUNED, 0, 0.0, 0, 0, plan["batch"])
    H.plan()
    bc.adaptive_source(H, torch.from_numpy(tg).to(dev), 2.0, 5, 300)
    if eff["schedule"] == bc.BC_SCHED_BATCHED:
        planned = plan["bottom_up"] if plan["bottom_up"] != 0 else 0.04
        assert H.stats()["bottom_up"] == planned
    H.close()
    G.close()


def test_round_thresholds_are_kept_per_width(dev):
    """The same handle's sampler at widths 256, 512 and 256 again: each width's
    threshold is one of the candidates, the second call at 256 reuses the
    first's, and the estimates equal the oracle's at every width."""
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    G = bc.Graph(g.row, g.col)
    plan = G.tune()
    tg = gg.top_degree(g, 3)
    want = O.adaptive_source(g, tg, 2.0, 5, 300)
    seen = {}
    for sb in (256, 512, 256):
        say("round threshold, width", sb)
        G.configure(bc.BC_SCHED_TUNED, 0, 0.0, 0, 0, sb)
        est = bc.adaptive_source(G, torch.from_numpy(tg).to(dev), 2.0, 5, 300)
        assert np.array_equal(est[1].cpu().numpy(), want[1])
        assert_close(est[0].cpu().numpy(), want[0], what="sampler at width %d" % sb)
        st = G.stats()
        assert st["batch_width"] == sb
        if G.plan()["schedule"] != bc.BC_SCHED_BATCHED:
            assert st["bottom_up"] == 0.0
            continue
        if sb == plan["batch"]:
            assert st["bottom_up"] == (plan["bottom_up"] if plan["bottom_up"] != 0 else 0.04)
        else:
            assert st["bottom_up"] in BOTTOM_UP
        if sb in seen:
            assert st["bottom_up"] == seen[sb]
        seen[sb] = st["bottom_up"]
    G.close()
