"""Full-size GPU parity in the benchmarks' launch configurations.

At these sizes the oracle cannot replay whole runs in seconds, so the checks
take outputs it can compute one at a time (sampled sources and pairs) and
properties that hold at any size (the per-vertex sum equals the sum of the
per-source rows; the per-source dependency sum equals the distance sum).
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402
from test_gpu_parity import assert_close, assert_sigma  # noqa: E402

O = oracle.load()


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ba(dev):
    g = gg.config_graph("ba1m")
    G = bc.Graph(g.row, g.col)
    yield g, G
    G.close()


def test_ba1m_bench_batch_sampled_rows(dev, ba):
    """The benchmark's step in its tuned plan: the 4096 sources (seed 7) as one
    batch of 64 words, bottom-up past 0.15 of the (vertex, word) entries. Rows
    0, 777, 2047 and 4095 against the oracle, every row's dependency sum
    against its distance sum, and the per-vertex sum (the benchmark's output)
    against the sum of all 4096 rows."""
    g, G = ba
    src = gg.philox_sources(7, 4096, g.n)
    t = torch.from_numpy(src).to(dev)
    G.configure(bc.BC_SCHED_BATCHED, 4096, 0.15)
    say("ba1m full rows, batch 4096")
    full, dist, _ = bc.dependencies(G, t, bc.BC_OUT_FULL, dist=True)
    assert G.stats()["batch_width"] == 4096 and G.stats()["schedule"] == bc.BC_SCHED_BATCHED
    for i in (0, 777, 2047, 4095):
        d, _, de = O.brandes(g, int(src[i]))
        assert np.array_equal(dist[i].cpu().numpy(), d), i
        got = full[i].cpu().numpy()
        assert_close(got, de, what="ba1m row %d" % i)
    # every source reaches all n vertices: its dependencies sum to the
    # distance sum minus the n - 1 targets' own terms
    rows = full.sum(1).cpu().numpy()
    dsum = (dist.sum(1, dtype=torch.int64) - (g.n - 1)).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(rows - dsum) <= 1e-9 * dsum)
    acc = full.sum(0)
    del full, dist
    say("ba1m sum, batch 4096")
    out, _, _ = bc.dependencies(G, t, bc.BC_OUT_SUM)
    assert_close(out.cpu().numpy(), acc.cpu().numpy(), rtol=1e-9, what="ba1m sum vs rows")
    G.configure(bc.BC_SCHED_AUTO, 0, 0.0)


def test_ba1m_pair_dependencies_from_the_stream(dev, ba):
    """Pairs 0, 1 and 5000 of the pair stream (seed 7), as the pair sampler
    draws them, against the oracle's two-search definition."""
    g, G = ba
    us = torch.empty(5001, dtype=torch.int32, device=dev)
    vs = torch.empty(5001, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 7, 0, 5001, us, vs)
    pick = [0, 1, 5000]
    u = us[pick].contiguous()
    v = vs[pick].contiguous()
    say("ba1m pairs")
    got = bc.pair_dependencies(G, u, v).cpu().numpy()
    for r, j in enumerate(pick):
        assert (int(u[r]), int(v[r])) == O.draw_pair(7, j, g.n)
        assert_close(got[r], O.pair_dependency(g, int(u[r]), int(v[r])), what="pair %d" % j)


@pytest.mark.parametrize("sched", [bc.BC_SCHED_AUTO, bc.BC_SCHED_WORKGROUP], ids=["auto", "wg"])
def test_grid2048_sampled_rows(dev, sched):
    """The percolated 2048^2 grid with its 1024 benchmark sources (seed 3):
    automatic schedule (pair-per-thread) and one workgroup per source, both
    with extended counts; rows 0 and 511 of the first 512 against the oracle,
    and the sum over those 512 against the sum of their rows."""
    g = gg.config_graph("grid2048")
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 0, 0.0)
    src = gg.philox_sources(3, 1024, g.n)
    t = torch.from_numpy(src[:512]).to(dev)
    say("grid2048 full", sched)
    full, dist, sig = bc.dependencies(G, t, bc.BC_OUT_FULL, dist=True, sigma=True)
    st = G.stats()
    want_sched = bc.BC_SCHED_THREADED if sched == bc.BC_SCHED_AUTO else sched
    assert st["schedule"] == want_sched and st["extended"] == 1
    for i in (0, 511):
        d, (om, oe), de = O.brandes(g, int(src[i]))
        assert np.array_equal(dist[i].cpu().numpy(), d)
        assert_sigma(sig[0][i].cpu().numpy(), sig[1][i].cpu().numpy(), om, oe, "grid row %d" % i)
        assert_close(full[i].cpu().numpy(), de, what="grid row %d" % i)
        assert (oe > 1024).any()           # counts beyond the FP64 range occur on this row
    del dist, sig
    say("grid2048 sum", sched)
    tot, _, _ = bc.dependencies(G, t, bc.BC_OUT_SUM)
    assert_close(tot.cpu().numpy(), full.sum(0).cpu().numpy(), rtol=1e-9, what="grid sum")
    G.close()


def test_rmat16_adaptive_source_hubs(dev):
    """C2's graph and batch width (256 per round), c = 5, seed 2, on its four
    highest-degree vertices (targets that stop after a few hundred samples)."""
    g = gg.config_graph("rmat16")
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_AUTO, 256, 0.0)
    targets = gg.top_degree(g, 4)
    say("rmat16 sampler")
    est, k, S, st = bc.adaptive_source(G, torch.from_numpy(targets).to(dev), 5.0, 2, g.n)
    oest, ok, oS, ost = O.adaptive_source(g, targets, 5.0, 2, g.n)
    assert np.array_equal(k.cpu().numpy(), ok) and np.array_equal(st.cpu().numpy(), ost)
    assert_close(est.cpu().numpy(), oest, what="rmat16 est")
    assert G.stats()["batch_width"] == 256
    G.close()
