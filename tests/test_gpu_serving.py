"""GPU tests of the query server (continuous batching over resident graphs).

A query's result must be bit-identical whether it runs alone or mixed with
other queries (on the same and on other graphs), and identical to the
single-target sampler calls with the same seed; sampled checks against the
oracle pin the values themselves.
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
GIB = 1 << 30


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


GRAPHS = [("er300", lambda: gg.er(300, 0.02, seed=5)),
          ("rmat10", lambda: gg.rmat(10, 8, 0.57, 0.19, 0.19, seed=2)),
          ("grid30", lambda: gg.grid(30, 30))]      # deep: served by the pair-per-thread engine


def make_queries(graphs):
    """(graph index, target, kind, rule, c, eps, seed, k_max) mixes."""
    qs = []
    r = np.random.default_rng(4)
    for gi, g in enumerate(graphs):
        tops = gg.top_degree(g, 3)
        for t in tops:
            qs.append((gi, int(t), bc.BC_QUERY_SOURCE, 0, float(r.choice([2.0, 5.0])), 0.1,
                       int(r.integers(1, 1 << 40)), g.n))
            qs.append((gi, int(t), bc.BC_QUERY_PAIR, bc.BC_PAIR_EPS, 1.0,
                       float(r.choice([0.1, 0.2])), int(r.integers(1, 1 << 40)), 1 << 16))
    leaf = int(np.flatnonzero(graphs[0].degree() == 1)[0])
    qs.append((0, leaf, bc.BC_QUERY_SOURCE, 0, 1.0, 0.1, 99, 50))   # capped at k_max
    qs.append((0, leaf, bc.BC_QUERY_PAIR, bc.BC_PAIR_ALG1, 1.0, 0.1, 98, 70))
    return qs


def new_server(graphs, budget=8 * GIB, max_batch=128):
    """A server holding `graphs` (ids 0, 1, ...)."""
    S = bc.Server(budget, max_batch)
    ids = [S.add_graph(g.row, g.col) for g in graphs]
    assert ids == list(range(len(graphs)))
    return S


def run(S, qs):
    ids = [S.submit(gi, t, kind, seed, kmax, c=c, eps=eps, rule=rule)
           for gi, t, kind, rule, c, eps, seed, kmax in qs]
    out = {}
    steps = 0
    while len(out) < len(qs):
        S.step()
        steps += 1
        assert steps < 100000
        for r in S.poll():
            out[r["id"]] = r
    return [out[i] for i in ids]


def key(r):
    return (r["est"], r["samples"], r["S"], r["status"])


def test_mixed_equals_alone_equals_sampler(dev):
    graphs = [m() for _, m in GRAPHS]
    qs = make_queries(graphs)
    say("serving mixed", len(qs))
    S = new_server(graphs)
    mixed = run(S, qs)
    st = S.stats()
    assert st["finished"] == len(qs) and st["queued"] == 0 and st["active"] == 0
    assert st["samples_used"] == sum(r["samples"] for r in mixed)
    S.close()
    for i, q in enumerate(qs):
        say("serving alone", i)
        A = new_server(graphs)
        alone = run(A, [q])[0]
        A.close()
        assert key(alone) == key(mixed[i]), (i, q, alone, mixed[i])
    # the same queries through the single-target sampler calls (pair samples
    # by the two-sided search, as the server runs them)
    for i, (gi, t, kind, rule, c, eps, seed, kmax) in enumerate(qs):
        g = graphs[gi]
        G = bc.Graph(g.row, g.col)
        tt = torch.tensor([t], dtype=torch.int32, device=dev)
        if kind == bc.BC_QUERY_SOURCE:
            est, k, Sx, stt = bc.adaptive_source(G, tt, c, seed, kmax)
        else:
            est, k, Sx, stt = bc.adaptive_pair(G, tt, rule, eps, c, seed, kmax)
        G.close()
        assert (est.item(), k.item(), Sx.item(), stt.item()) == key(mixed[i]), (i, q)


def test_serving_against_oracle(dev):
    g = gg.er(300, 0.02, seed=5)
    S = new_server([g])
    tops = gg.top_degree(g, 2)
    qs = [(0, int(tops[0]), bc.BC_QUERY_SOURCE, 0, 3.0, 0.1, 17, g.n),
          (0, int(tops[1]), bc.BC_QUERY_PAIR, bc.BC_PAIR_EPS, 1.0, 0.15, 23, 1 << 16)]
    say("serving oracle")
    res = run(S, qs)
    S.close()
    oe, ok, oS, ost = O.adaptive_source(g, [tops[0]], 3.0, 17, g.n)
    assert res[0]["samples"] == ok[0] and res[0]["status"] == ost[0]
    assert abs(res[0]["est"] - oe[0]) <= 1e-9 * oe[0]
    oe, ok, oS, ost = O.adaptive_pair(g, [tops[1]], oracle.RULE_EPS, 0.15, 1.0, 23, 1 << 16)
    assert res[1]["samples"] == ok[0] and res[1]["status"] == ost[0]
    assert abs(res[1]["est"] - oe[0]) <= 1e-9 * oe[0]


def test_continuous_admission_and_latency_fields(dev):
    graphs = [gg.er(300, 0.02, seed=5), gg.rmat(10, 8, 0.57, 0.19, 0.19, seed=2)]
    S = new_server(graphs, max_batch=64)
    say("serving continuous")
    t0 = S.now()
    first = [S.submit(0, int(gg.top_degree(graphs[0], 1)[0]), bc.BC_QUERY_PAIR, 7 + i, 1 << 16,
                      eps=0.1, rule=bc.BC_PAIR_EPS) for i in range(3)]
    S.step()
    # arrivals while the first queries are active join later rounds
    later = [S.submit(i % 2, int(gg.top_degree(graphs[i % 2], 2)[1]), bc.BC_QUERY_SOURCE,
                      50 + i, 5000, c=2.0) for i in range(6)]
    got = {}
    while len(got) < 9:
        S.step()
        for r in S.poll():
            got[r["id"]] = r
    for i in first + later:
        r = got[i]
        assert r["done_s"] >= r["arrival_s"] >= t0
    st = S.stats()
    assert st["rounds"] >= 2 and st["samples_executed"] >= st["samples_used"]
    S.close()


def test_budget_admission(dev):
    g = gg.er(2000, 0.004, seed=1)
    say("serving budget")
    S = bc.Server(1 << 12, 64)             # 4 KiB: the CSR itself does not fit
    with pytest.raises(bc.BcError) as e:
        S.add_graph(g.row, g.col)
    assert e.value.status == bc.BC_E_NOMEM
    S.close()
    S = bc.Server(200 << 10, 64)           # CSR fits, no engine workspace does
    with pytest.raises(bc.BcError) as e:
        S.add_graph(g.row, g.col)
    assert e.value.status == bc.BC_E_NOMEM
    S.close()
    S = bc.Server(8 * GIB, 64)
    gid = S.add_graph(g.row, g.col)
    with pytest.raises(bc.BcError):
        S.submit(gid + 1, 0, bc.BC_QUERY_SOURCE, 1, 10, c=2.0)
    with pytest.raises(bc.BcError):
        S.submit(gid, 2000, bc.BC_QUERY_SOURCE, 1, 10, c=2.0)
    with pytest.raises(bc.BcError):
        S.submit(gid, 0, bc.BC_QUERY_PAIR, 1, 10, eps=0.7, rule=bc.BC_PAIR_EPS)
    assert S.step() == 0                   # nothing queued: no device work
    S.close()


def test_widest_batch_mixed_alone_oracle(dev):
    """max_batch 4096: the shallow graph runs 64-word wave batches, the deep
    one 4096-lane pair-engine batches. Mixed = alone = oracle."""
    graphs = [gg.rmat(10, 8, 0.57, 0.19, 0.19, seed=2), gg.grid(40, 40)]
    qs = []
    for gi, g in enumerate(graphs):
        for j, t in enumerate(gg.top_degree(g, 2)):
            qs.append((gi, int(t), bc.BC_QUERY_SOURCE, 0, 2.0, 0.1, 31 + 7 * j + gi, 1024))
            qs.append((gi, int(t), bc.BC_QUERY_PAIR, bc.BC_PAIR_EPS, 1.0, 0.1, 61 + 5 * j + gi,
                       4096))
    say("serving max_batch 4096 mixed", len(qs))
    S = new_server(graphs, budget=32 * GIB, max_batch=4096)
    assert S.graph_width(0) == (4096, bc.BC_SCHED_BATCHED)
    assert S.graph_width(1) == (4096, bc.BC_SCHED_THREADED)
    mixed = run(S, qs)
    st = S.stats()
    assert st["resident_bytes"] + st["workspace_bytes"] <= st["budget_bytes"]
    S.close()
    for i, q in enumerate(qs):
        say("serving max_batch 4096 alone", i)
        A = new_server(graphs, budget=32 * GIB, max_batch=4096)
        alone = run(A, [q])[0]
        A.close()
        assert key(alone) == key(mixed[i]), (i, q)
        gi, t, kind, rule, c, eps, seed, kmax = q
        g = graphs[gi]
        if kind == bc.BC_QUERY_SOURCE:
            oe, ok, oS, ost = O.adaptive_source(g, [t], c, seed, kmax)
        else:
            oe, ok, oS, ost = O.adaptive_pair(g, [t], oracle.RULE_EPS, eps, c, seed, kmax)
        assert mixed[i]["samples"] == ok[0] and mixed[i]["status"] == ost[0], (i, q)
        assert abs(mixed[i]["est"] - oe[0]) <= 1e-9 * abs(oe[0]), (i, q)


def test_budget_is_an_invariant(dev):
    """Graph after graph, and round after round, resident bytes plus the shared
    workspace stay within the budget; a tight budget narrows the widths."""
    graphs = [gg.rmat(s, 8, 0.57, 0.19, 0.19, seed=40 + s) for s in (11, 13, 12)] + \
             [gg.grid(70, 70)]
    budget = 96 << 20
    say("serving budget invariant")
    S = bc.Server(budget, 4096)
    for g in graphs:
        S.add_graph(g.row, g.col)
        st = S.stats()
        assert st["resident_bytes"] + st["workspace_bytes"] <= budget
    widths = [S.graph_width(i)[0] for i in range(len(graphs))]
    assert min(widths) < 4096, widths
    qs = []
    for gi, g in enumerate(graphs):
        t = int(gg.top_degree(g, 1)[0])
        qs.append((gi, t, bc.BC_QUERY_SOURCE, 0, 2.0, 0.1, 5 + gi, 600))
        qs.append((gi, t, bc.BC_QUERY_PAIR, bc.BC_PAIR_EPS, 1.0, 0.2, 9 + gi, 2000))
    for gi, t, kind, rule, c, eps, seed, kmax in qs:
        S.submit(gi, t, kind, seed, kmax, c=c, eps=eps, rule=rule)
    done = 0
    while done < len(qs):
        S.step()
        done += len(S.poll())
        st = S.stats()
        assert st["resident_bytes"] + st["workspace_bytes"] <= budget, st
    S.close()
    # a budget that holds the graphs but not the widest width gets narrower
    # widths, never a larger footprint
    S = bc.Server(32 << 20, 4096)
    S.add_graph(graphs[1].row, graphs[1].col)
    assert S.graph_width(0)[0] < widths[1] or widths[1] == 64
    st = S.stats()
    assert st["resident_bytes"] + st["workspace_bytes"] <= 32 << 20
    S.close()


def test_rounds_split_when_the_record_outgrows_the_budget(dev):
    """A hub with 1100 paths of 15 vertices: shallow from the hub (wave
    engine), but a word of random sources meets each vertex at ~15 levels, far
    beyond the 4 record entries per (vertex, word) a server budgets. Rounds
    then run their samples in halves; results match the oracle."""
    paths, length = 1100, 15
    n = 1 + paths * length
    src, dst = [], []
    for p in range(paths):
        first = 1 + p * length
        src.append(0)
        dst.append(first)
        for i in range(length - 1):
            src.append(first + i)
            dst.append(first + i + 1)
    g = gg.from_edges(n, src, dst, "broom")
    qs = [(0, 0, bc.BC_QUERY_SOURCE, 0, 2.0, 0.1, 3, 64),
          (0, 1 + 3 * length + 4, bc.BC_QUERY_SOURCE, 0, 1.5, 0.1, 4, 64)]
    say("serving split rounds")
    S = new_server([g], budget=GIB, max_batch=64)
    assert S.graph_width(0) == (64, bc.BC_SCHED_BATCHED)
    res = run(S, qs)
    st = S.stats()
    assert st["split_rounds"] > 0, st
    assert st["resident_bytes"] + st["workspace_bytes"] <= GIB
    S.close()
    for i, (gi, t, kind, rule, c, eps, seed, kmax) in enumerate(qs):
        oe, ok, oS, ost = O.adaptive_source(g, [t], c, seed, kmax)
        assert res[i]["samples"] == ok[0] and res[i]["status"] == ost[0]
        assert abs(res[i]["est"] - oe[0]) <= 1e-9 * abs(oe[0])


def test_lanes_equal_one_lane(dev):
    """Rounds of up to four graphs at once (one stream and workspace per
    lane): every query's result equals the one-lane server's, bit for bit;
    the budget holds one workspace per lane."""
    graphs = [m() for _, m in GRAPHS] + [gg.rmat(9, 8, 0.57, 0.19, 0.19, seed=7),
                                         gg.er(500, 0.01, seed=3)]
    qs = make_queries(graphs)
    say("serving one lane", len(qs))
    S = new_server(graphs)
    one = run(S, qs)
    S.close()
    for lanes in (2, 4):
        say("serving lanes", lanes)
        S = new_server(graphs)
        S.set_lanes(lanes)
        got = run(S, qs)
        st = S.stats()
        assert st["resident_bytes"] + st["workspace_bytes"] <= st["budget_bytes"]
        assert st["finished"] == len(qs)
        S.close()
        for i in range(len(qs)):
            assert key(got[i]) == key(one[i]), (lanes, i, qs[i], got[i], one[i])


def test_lanes_budget(dev):
    """Lanes need one workspace each within the budget: some budget admits
    the graph with one lane but refuses four; a large one takes four."""
    g = gg.er(2000, 0.004, seed=1)
    say("serving lanes budget")
    refused = False
    for kib in (256, 384, 512, 768, 1024, 1536, 2048, 4096, 8192):
        S = bc.Server(kib << 10, 64)
        try:
            S.add_graph(g.row, g.col)
        except bc.BcError as e:
            assert e.status == bc.BC_E_NOMEM
            S.close()
            continue
        try:
            S.set_lanes(4)
        except bc.BcError as e:
            assert e.status == bc.BC_E_INVALID
            refused = True
            S.set_lanes(1)
            S.close()
            break
        S.close()
    assert refused
    S = bc.Server(8 * GIB, 64)
    S.add_graph(g.row, g.col)
    S.set_lanes(4)
    with pytest.raises(bc.BcError):
        S.set_lanes(5)
    S.set_lanes(2)
    S.close()


def diamond_chain(d):
    """Vertex 0, then d diamonds: c_{i-1} -> a_i, b_i -> c_i (c_0 = 0), so
    sigma(0, c_i) = 2^i and pairs more than ~1000 diamonds apart have path
    counts beyond 2^1000."""
    src, dst = [], []
    prev = 0
    for i in range(d):
        a, b, c = 1 + 3 * i, 2 + 3 * i, 3 + 3 * i
        src += [prev, prev, a, b]
        dst += [a, b, c, c]
        prev = c
    return gg.from_edges(1 + 3 * d, np.array(src), np.array(dst), "diamonds%d" % d)


def test_pair_queries_past_the_fp64_range(dev):
    """Pair slots run on the two-sided search, which works in plain FP64: once
    a round meets a pair whose path count reaches 2^1000, that round's pair
    slots and the graph's later ones run one-sided (extended counts). Both
    queries still match the oracle."""
    g = diamond_chain(1100)
    qs = [(0, 3, bc.BC_QUERY_PAIR, bc.BC_PAIR_EPS, 1.0, 0.1, 41, 1500),   # capped at k_max
          (0, 3 * 550 - 1, bc.BC_QUERY_SOURCE, 0, 2.0, 0.1, 43, 200)]
    G = bc.Graph(g.row, g.col)
    u = torch.empty(1500, dtype=torch.int32, device=dev)
    v = torch.empty(1500, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 41, 0, 1500, u, v)
    G.close()
    apart = np.abs((u.cpu().numpy() - 1) // 3 - (v.cpu().numpy() - 1) // 3)
    assert (apart > 1010).sum() >= 3       # some drawn pairs count beyond 2^1000
    say("serving diamond chain")
    S = new_server([g], budget=8 * GIB, max_batch=512)
    res = run(S, qs)
    S.close()
    oe, ok, oS, ost = O.adaptive_pair(g, [3], oracle.RULE_EPS, 0.1, 1.0, 41, 1500)
    assert res[0]["samples"] == ok[0] == 1500 and res[0]["status"] == ost[0], (res[0], ok, ost)
    assert abs(res[0]["est"] - oe[0]) <= 1e-9 * abs(oe[0])
    oe, ok, oS, ost = O.adaptive_source(g, [3 * 550 - 1], 2.0, 43, 200)
    assert res[1]["samples"] == ok[0] and res[1]["status"] == ost[0]
    assert abs(res[1]["est"] - oe[0]) <= 1e-9 * abs(oe[0])
