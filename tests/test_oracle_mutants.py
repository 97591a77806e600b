"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle.c, applies one plausible slip (a dropped term, a
wrong level, a wrong comparison, a wrong constant), builds it on the CPU, and
runs a compact selection of the pins from test_oracle_*.py against it. The
unmodified source must pass the same selection.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import networkx as nx
import pytest

import graphgen as gg
import oracle
from bruteforce import Brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "oracle.h")

MUTANTS = {
    "drop_one_in_recursion": ("double r = 1.0 + p->delta[t];", "double r = p->delta[t];"),
    "sigma_from_same_level": ("if (p->dist[u] == p->dist[w] - 1) acc",
                              "if (p->dist[u] == p->dist[w]) acc"),
    "successor_level_wrong": ("if (p->dist[t] == p->dist[v] + 1) {",
                              "if (p->dist[t] >= p->dist[v] && t != v) {"),
    "source_keeps_own_dependency": ("for (int64_t i = p->reached - 1; i >= 1; --i)",
                                    "for (int64_t i = p->reached - 1; i >= 0; --i)"),
    "ratio_inverted": ("double q = xnum_div(p->sig[v], p->sig[t]);",
                       "double q = xnum_div(p->sig[t], p->sig[v]);"),
    "stop_on_equal": ("if (S[i] > threshold) { status[i] = ST_DONE;",
                      "if (S[i] >= threshold) { status[i] = ST_DONE;"),
    "pair_shift_missing": ("if (b >= a) b += 1;", "if (b > a) b += 1;"),
    "source_range_excludes_one": ("return (int32_t)scale_draw(w[0], n);",
                                  "return (int32_t)scale_draw(w[0], n - 1);"),
    "estimate_scale_wrong": ("est[i] = ((double)n * S[i]) / (double)samples[i];",
                             "est[i] = ((double)(n - 1) * S[i]) / (double)samples[i];"),
    "philox_nine_rounds": ("for (int r = 0; r < 10; ++r) {", "for (int r = 0; r < 9; ++r) {"),
    "philox_key_bump_swapped": ("k0 += W0; k1 += W1;", "k0 += W1; k1 += W0;"),
    "exponent_align_wrong": ("ldexp(a.m, a.e - e) + ldexp(b.m, b.e - e)",
                             "ldexp(a.m, a.e - e) + ldexp(b.m, e - b.e)"),
    "pair_offpath_kept": ("if (pu->dist[t] + pv->dist[t] != duv) continue;",
                          "if (pu->dist[t] + pv->dist[t] > duv + 1) continue;"),
    "eps_rule_unsquared": ("((double)samples[i] * (S[i] * S[i])) >= eps_rhs",
                           "((double)samples[i] * S[i]) >= eps_rhs"),
    "pair_estimate_scale": ("const double pairs = (double)n * (double)(n - 1);",
                            "const double pairs = (double)n * (double)n;"),
}


# slips in the work counters (the throughput metric's numerators)
WORK_MUTANTS = {
    "dag_counts_same_level": ("if (p.dist[col[e]] == p.dist[u] + 1) ++dag;",
                              "if (p.dist[col[e]] >= p.dist[u] && col[e] != u) ++dag;"),
    "component_edges_doubled": ("*edges_undirected = deg / 2;", "*edges_undirected = deg;"),
    "pair_limit_inclusive": ("if (lead && da < limit) ++cnt;", "if (lead && da <= limit) ++cnt;"),
    "pair_same_level_twice": ("int lead = (da < db) || (da == db && a < b);",
                              "int lead = (da <= db);"),
    "reached_without_source": ("if (reached) *reached = p.reached;",
                               "if (reached) *reached = p.reached - 1;"),
    "bidir_ties_to_side_one": ("const int s = vol[0] <= vol[1] ? 0 : 1, o = 1 - s;",
                               "const int s = vol[0] < vol[1] ? 0 : 1, o = 1 - s;"),
    "bidir_frontier_by_vertices": ("nv += row[s][y + 1] - row[s][y];", "nv += 1;"),
    "bidir_counts_every_new_vertex": ("if (!meet || dist[o][w] >= 0) na += row[o][w + 1] - row[o][w];",
                                      "na += row[o][w + 1] - row[o][w];"),
    "bidir_sweep_stops_above_level_zero": ("for (int L = depth[s] - 1; L >= 0; --L) {",
                                           "for (int L = depth[s] - 1; L >= 1; --L) {"),
    "bidir_sweep_pull_wrong_direction": ("if (dist[o][w] == D - L) na += row[s][w + 1] - row[s][w];",
                                         "if (dist[o][w] == D - L) na += row[o][w + 1] - row[o][w];"),
}


def build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    d = tmp_path / name
    d.mkdir()
    shutil.copy(HDR, d / "oracle.h")
    (d / "oracle.c").write_text(src.replace(old, new))
    out = str(d / "lib.so")
    subprocess.check_call(["gcc"] + oracle.CFLAGS + [str(d / "oracle.c"), "-o", out, "-lm"])
    return oracle.load(out)


def numpy_block(seed, stream, j):
    c = (j - 1) % (1 << 256)
    ctr = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64), counter=ctr)
    return [int(x) for x in bg.random_raw(4)]


def pins_pass(O):
    """A compact selection of the pins; True when all of them hold."""
    try:
        # Philox and the draw maps against numpy
        if [int(x) for x in O.philox([5, 0, 0, 0], [7, 0])] != numpy_block(7, 0, 5):
            return False
        for j in range(20):
            w = numpy_block(3, 0, j)
            if O.draw_source(3, j, 10) != (w[0] * 10) >> 64:
                return False
            w = numpy_block(3, 1, j)
            u = (w[0] * 10) >> 64
            v = (w[1] * 9) >> 64
            if O.draw_pair(3, j, 10) != (u, v + (v >= u)):
                return False
        # brute force on small graphs
        for G in nx.graph_atlas_g()[40:1253:37]:
            n = G.number_of_nodes()
            e = np.array(list(G.edges()), dtype=np.int64).reshape(-1, 2)
            g = gg.from_edges(n, e[:, 0], e[:, 1])
            b = Brute(g)
            bc = O.bc_exact(g)
            if not np.allclose(bc, [float(x) for x in b.bc()], rtol=1e-12, atol=1e-12):
                return False
            for u in range(n):
                for v in range(n):
                    if u != v:
                        y = O.pair_dependency(g, u, v)
                        if not np.allclose(y, [float(x) for x in b.pair_dep(u, v)],
                                           rtol=1e-12, atol=1e-12):
                            return False
        # grid counts beyond the FP64 range
        g = gg.grid(600, 600)
        dist, (sm, se), de = O.brandes(g, 0)
        for i, j in ((599, 599), (599, 3), (300, 200)):
            v = i * 600 + j
            got = Fraction(float(sm[v])) * Fraction(2) ** int(se[v])
            want = math.comb(i + j, i)
            if abs(got - want) > Fraction(want, 10 ** 12):
                return False
        # sampler loops: star closed form, path tie, EPS rule on a star
        n, c, seed = 10, 3.0, 2
        S, k = 0, 0
        for j in range(4000):
            s = (numpy_block(seed, 0, j)[0] * n) >> 64
            S += 0 if s == 0 else n - 2
            k += 1
            if S > c * n:
                break
        est, kk, SS, st = O.adaptive_source(gg.star(n), [0], c, seed, 10 ** 6)
        if (kk[0], SS[0], st[0], est[0]) != (k, S, 0, n * S / k):
            return False
        for seed in range(1, 6):
            _, kk, SS, _ = O.adaptive_source(gg.path(5), [2], 2.0, seed, 10 ** 6)
            if SS[0] != 12:
                return False
        for n, eps, seed in ((9, 0.1, 3), (30, 0.2, 4)):
            S, k = 0, 0
            for j in range(100000):
                w = numpy_block(seed, 1, j)
                u = (w[0] * n) >> 64
                v = (w[1] * (n - 1)) >> 64
                v += v >= u
                S += 1 if (u != 0 and v != 0) else 0
                k += 1
                if S > 0 and k * S * S >= eps ** 3 * n * n:
                    break
            est, kk, SS, st = O.adaptive_pair(gg.star(n), [0], 1, eps, 1.0, seed, 10 ** 7)
            if (kk[0], SS[0]) != (k, S) or est[0] != n * (n - 1) * S / k:
                return False
    except ValueError:
        return False
    return True


def work_pins_pass(O):
    """A compact selection of the work-counter pins (tests/test_oracle_work.py)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    try:
        if O.source_work(gg.cycle(7), 0) != (7, 7, 6):
            return False
        if O.source_work(gg.grid(5, 9), 0) != (45, 76, 76):
            return False
        g = gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6])
        if O.source_work(g, 0) != (3, 3, 2) or O.pair_work(g, 0, 5) != 3:
            return False
        n = 12
        p = gg.path(n)
        for u, v in ((0, 5), (7, 2), (3, 4)):
            k = abs(u - v)
            if O.pair_work(p, u, v) != min(u, k) + min(k, n - 1 - u):
                return False
        # the two-sided search's walks, worked by hand (tests/test_oracle_work.py)
        if O.bidir_work(gg.star(6), 1, 2) != (2, 24) or O.bidir_work(gg.star(6), 0, 1) != (1, 12):
            return False
        if O.bidir_work(gg.path(9), 0, 8) != (8, 60):
            return False
        if O.bidir_work(gg.directed_path(5), 0, 4, directed=True) != (4, 16):
            return False
        if O.bidir_work(gg.from_edges(8, [0, 1, 0, 3, 4, 5], [1, 2, 2, 4, 5, 6]), 0, 5) != (5, 16):
            return False
        if O.bidir_work(gg.from_edges(5, [0, 0, 1, 2], [1, 2, 3, 4]), 0, 1) != (2, 8):
            return False
        if O.bidir_work(gg.from_edges(4, [0, 3, 1], [3, 1, 2]), 0, 1) != (2, 14):
            return False
        g = gg.er(300, 0.012, seed=3)
        a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row), shape=(g.n, g.n))
        src = np.repeat(np.arange(g.n), np.diff(g.row))
        dst = g.col.astype(np.int64)
        for u, v in ((0, 1), (5, 200), (17, 299)):
            d = shortest_path(a, unweighted=True, directed=False, indices=[u])[0]
            d = np.where(np.isinf(d), -1, d).astype(np.int64)
            dag = int(((d[src] >= 0) & (d[dst] == d[src] + 1)).sum())
            if O.source_work(g, u) != (int((d >= 0).sum()), int((d[src] >= 0).sum()) // 2, dag):
                return False
            lim = d[v] if d[v] >= 0 else 1 << 40
            keep = src < dst
            da, db = d[src[keep]], d[dst[keep]]
            if O.pair_work(g, u, v) != int(((da >= 0) & (np.minimum(da, db) < lim)).sum()):
                return False
    except ValueError:
        return False
    return True


def test_unmodified_oracle_passes_the_selection():
    O = oracle.load()
    assert pins_pass(O)
    assert work_pins_pass(O)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert not pins_pass(build_variant(tmp_path, name, old, new))


@pytest.mark.parametrize("name", sorted(WORK_MUTANTS))
def test_planted_work_counter_mistake_is_caught(tmp_path, name):
    old, new = WORK_MUTANTS[name]
    assert not work_pins_pass(build_variant(tmp_path, name, old, new))
