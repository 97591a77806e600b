"""Brute-force betweenness by explicit shortest-path enumeration, exact rationals.

Independent of the oracle: every simple path between every ordered pair is
enumerated by depth-first search, the shortest ones (fewest arcs, or least
total weight when the graph carries arc weights g.w) are kept, and the
definitions (pair dependency sigma_st(v)/sigma_st, Definition 1; source
dependency, Definition 2) are evaluated on them with fractions.Fraction. Meant
for graphs of at most a dozen sparse vertices.
"""
from __future__ import annotations

from fractions import Fraction


def adjacency(g):
    """[(head, length)] per vertex: length 1, or the arc's weight."""
    w = getattr(g, "w", None)
    return [[(int(g.col[e]), 1 if w is None else int(w[e])) for e in range(g.row[v], g.row[v + 1])]
            for v in range(g.n)]


def shortest_paths_from(adj, s):
    """dict t -> (length, list of shortest s-t paths as tuples), over all
    simple paths."""
    best = {}
    n = len(adj)
    on = [False] * n
    path = [s]
    on[s] = True

    def dfs(u, L0):
        for w, c in adj[u]:
            if on[w]:
                continue
            path.append(w)
            on[w] = True
            L = L0 + c
            cur = best.get(w)
            if cur is None or L < cur[0]:
                best[w] = [L, [tuple(path)]]
            elif L == cur[0]:
                cur[1].append(tuple(path))
            dfs(w, L)
            on[w] = False
            path.pop()

    dfs(s, 0)
    best.pop(s, None)
    return {t: (v[0], v[1]) for t, v in best.items()}


class Brute:
    def __init__(self, g):
        self.n = g.n
        self.adj = adjacency(g)
        self.paths = [shortest_paths_from(self.adj, s) for s in range(g.n)]

    def dist(self, s):
        d = [-1] * self.n
        d[s] = 0
        for t, (L, _) in self.paths[s].items():
            d[t] = L
        return d

    def sigma(self, s):
        sg = [0] * self.n
        sg[s] = 1
        for t, (_, ps) in self.paths[s].items():
            sg[t] = len(ps)
        return sg

    def pair_dep(self, s, t):
        """Fraction sigma_st(v)/sigma_st for every v (0 for v in {s, t})."""
        out = [Fraction(0)] * self.n
        if t not in self.paths[s]:
            return out
        ps = self.paths[s][t][1]
        tot = len(ps)
        for p in ps:
            for v in p[1:-1]:
                out[v] += Fraction(1, tot)
        return out

    def source_dep(self, s):
        out = [Fraction(0)] * self.n
        for t in self.paths[s]:
            for v, x in enumerate(self.pair_dep(s, t)):
                out[v] += x
        return out

    def bc(self):
        out = [Fraction(0)] * self.n
        for s in range(self.n):
            for v, x in enumerate(self.source_dep(s)):
                out[v] += x
        return out
