"""Parity on the configured workloads' own settings (graphs, targets, rules,
batch widths), with the sample cap lowered where the oracle would otherwise
run for minutes. Sample counts and statuses compare exactly, sums and
estimates within 1e-9 relative (Section 4's loop; Algorithm 1).

  C1  ER n = 2000: Algorithm 1 as printed (c = 1) on the highest-BC vertices
  C2  R-MAT scale 16: targets at degree percentiles, low-BC ones included,
      c = 5, 256 samples per round
  C3  BA n = 2^20: pair sampling, eps = 0.05, top-degree targets, 256 per round
  wave engine at its widest batch (4096 sources, 64 words) on R-MAT scale 12
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1608_04472_amd as bc  # noqa: E402
from test_gpu_parity import assert_close, check_sampler  # noqa: E402

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
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def test_c1_algorithm1_literal_rule(dev):
    g = gg.config_graph("er2000")
    bcx = O.bc_exact(g)
    tg = np.argsort(-bcx, kind="stable")[:4].astype(np.int32)
    G = bc.Graph(g.row, g.col)
    say("C1 ALG1 c=1")
    got = bc.adaptive_pair(G, T(tg, dev), bc.BC_PAIR_ALG1, 0.1, 1.0, 1, 10000)
    want = O.adaptive_pair(g, tg, oracle.RULE_ALG1, 0.1, 1.0, 1, 10000)
    check_sampler(got, want, "C1 alg1")
    G.close()


def test_c2_percentile_targets_low_and_high(dev):
    g = gg.config_graph("rmat16")
    tg64 = gg.degree_percentile_targets(g, 64)
    # five of the configured percentile targets (lowest to highest) and the
    # top hub, which stops within the cap
    tg = np.concatenate([tg64[[0, 18, 36, 54, 63]], gg.top_degree(g, 1)]).astype(np.int32)
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_AUTO, 256, 0.0)
    say("C2 percentiles c=5 B=256 k_max=400")
    got = bc.adaptive_source(G, T(tg, dev), 5.0, 2, 400)
    assert G.stats()["batch_width"] == 256
    want = O.adaptive_source(g, tg, 5.0, 2, 400)
    check_sampler(got, want, "C2 percentiles")
    assert (want[3] == oracle.CAPPED).any() and (want[3] == oracle.DONE).any()
    G.close()


def test_c3_pair_sampling_targets(dev):
    g = gg.config_graph("ba1m")
    tg = gg.top_degree(g, 32)[[0, 13, 31]]
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_AUTO, 256, 0.0)
    say("C3 pair eps=0.05 k_max=40")
    got = bc.adaptive_pair(G, T(tg, dev), bc.BC_PAIR_EPS, 0.05, 1.0, 7, 40)
    want = O.adaptive_pair(g, tg, oracle.RULE_EPS, 0.05, 1.0, 7, 40)
    check_sampler(got, want, "C3 pairs")
    assert np.all(want[2] > 0)
    G.close()


def test_wave_engine_widest_batch(dev):
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    src = gg.philox_sources(12, 4200, g.n)       # one full batch of 4096 and a ragged tail
    src[4100] = src[5] = src[4095]
    G = bc.Graph(g.row, g.col)
    G.configure(bc.BC_SCHED_BATCHED, 4096, 0.0)
    say("wave B=4096 k=4200")
    full, dist, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True)
    st = G.stats()
    assert st["batch_width"] == 4096 and st["batches"] == 2
    want, _ = O.dependencies(g, src, full=True, total=False)
    assert_close(full.cpu().numpy(), want, what="B=4096 rows")
    for i in (0, 4095, 4199):
        assert np.array_equal(dist[i].cpu().numpy(), O.brandes(g, int(src[i]))[0])
    say("wave B=4096 sum")
    tot, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_SUM)
    assert_close(tot.cpu().numpy(), want.sum(0), what="B=4096 sum")
    G.close()
