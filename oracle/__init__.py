"""CPU oracle for sampled betweenness centrality -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct C (oracle.c) with this ctypes wrapper. Only
tests/, the smoke check and the benchmark's CPU-baseline leg may import it;
the GPU library never loads it and shares no code with it.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
  philox4x64_10       numpy.random.Philox raw stream (independent code)
  brandes             brute-force path enumeration, closed forms, invariants,
                      networkx, scipy distances, binomial path counts on grids
  bc_exact            brute force, closed forms, sum invariant, networkx
  dependencies        same as brandes (it is a loop over brandes)
  pair_dependency     brute-force path enumeration; sum over all ordered pairs
                      equals BC; per-pair sum equals d(u,v)-1
  adaptive_source     closed form on a star, threshold tie on a path, capped
                      run on a leaf, target sharing, fixed-k unbiasedness.
                      Accuracy of the adaptive estimate itself: parity unpinned
  adaptive_pair       same checks as adaptive_source on its own rules.
                      Accuracy of the adaptive estimate: parity unpinned
  source_work         closed forms (paths, stars, cycles, complete, bipartite,
                      grids, trees), scipy BFS distances with numpy edge
                      counts, planted mistakes
  pair_work           closed forms (paths, stars, adjacent and unreachable
                      pairs), scipy BFS distances, planted mistakes
  bidir_work          the two-sided search's walks (the library's design, a
                      measurement check): closed forms worked by hand (stars,
                      paths, directed paths, unreachable pairs), bounds by
                      the components' sizes and arcs, planted mistakes
  *_weighted          the same functions on graphs with positive integer arc
                      weights (Dijkstra's algorithm): brute-force enumeration
                      of weighted shortest paths, networkx's weighted
                      betweenness, unit weights equal the unweighted oracle,
                      scaled weights leave every result unchanged, a weight
                      that lengthens an edge past a detour removes it from
                      every shortest path, planted mistakes
  *_directed          the same functions on directed graphs (out-neighbour
                      CSR): brute-force path enumeration on small digraphs,
                      closed forms (directed paths, cycles, stars, DAG
                      layers), networkx's directed betweenness, bidirected
                      graphs equal to their undirected form, planted mistakes
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]
_lib = None

RULE_ALG1 = 0
RULE_EPS = 1
DONE = 0
CAPPED = 1

_i64p = ctypes.c_void_p


def build(force: bool = False, extra_flags=None, out: str | None = None) -> str:
    """Compile oracle.c with gcc. extra_flags/out serve the mutation tests."""
    out = out or LIB_PATH
    if force or not os.path.exists(out) or extra_flags:
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc"] + CFLAGS + list(extra_flags or []) + [os.path.join(_HERE, "oracle.c"),
                                                              "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def _declare(lib):
    c = ctypes
    lib.oracle_philox4x64_10.restype = None
    lib.oracle_philox4x64_10.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p]
    lib.oracle_brandes.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_int32,
                                   c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.oracle_bc_exact.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.oracle_dependencies.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p,
                                        c.c_int64, c.c_void_p, c.c_void_p]
    lib.oracle_pair_dependency.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_int32,
                                           c.c_int32, c.c_void_p]
    lib.oracle_draw_source.restype = c.c_int32
    lib.oracle_draw_source.argtypes = [c.c_uint64, c.c_int64, c.c_int64]
    lib.oracle_draw_pair.restype = None
    lib.oracle_draw_pair.argtypes = [c.c_uint64, c.c_int64, c.c_int64, c.c_void_p, c.c_void_p]
    lib.oracle_adaptive_source.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p,
                                           c.c_int32, c.c_double, c.c_uint64, c.c_int64,
                                           c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    lib.oracle_adaptive_pair.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_void_p,
                                         c.c_int32, c.c_int, c.c_double, c.c_double,
                                         c.c_uint64, c.c_int64, c.c_void_p, c.c_void_p,
                                         c.c_void_p, c.c_void_p]
    lib.oracle_source_work.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_int32,
                                       c.c_void_p, c.c_void_p, c.c_void_p]
    lib.oracle_pair_work.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_int32,
                                     c.c_int32, c.c_void_p]
    lib.oracle_bidir_work.argtypes = [c.c_int64, c.c_void_p, c.c_void_p, c.c_int, c.c_int32,
                                      c.c_int32, c.c_void_p, c.c_void_p]
    lib.oracle_bidir_work.restype = c.c_int
    for name in ("oracle_brandes", "oracle_bc_exact", "oracle_dependencies",
                 "oracle_pair_dependency", "oracle_adaptive_source", "oracle_adaptive_pair"):
        d = getattr(lib, name + "_directed")
        d.argtypes = getattr(lib, name).argtypes
        w = getattr(lib, name + "_weighted")
        a = getattr(lib, name).argtypes
        w.argtypes = a[:3] + [c.c_void_p, c.c_int] + a[3:]
        w.restype = c.c_int
    for name in ("oracle_brandes", "oracle_bc_exact", "oracle_dependencies",
                 "oracle_pair_dependency", "oracle_adaptive_source", "oracle_adaptive_pair",
                 "oracle_source_work", "oracle_pair_work"):
        getattr(lib, name).restype = c.c_int
        if hasattr(lib, name + "_directed"):
            getattr(lib, name + "_directed").restype = c.c_int
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it if absent). A custom path loads a
    separately built variant without touching the cached default."""
    global _lib
    if path is not None:
        return Oracle(_declare(ctypes.CDLL(path)))
    if _lib is None:
        build()
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return Oracle(_lib)


def _p(a):
    return None if a is None else a.ctypes.data


def _csr(g):
    row = np.ascontiguousarray(g.row, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    return g.n, row, col


def _ok(rc, what):
    if rc != 0:
        raise ValueError("%s failed (rc=%d)" % (what, rc))


class Oracle:
    """Calls take an undirected CSR, or with directed=True a CSR of
    out-neighbours (edges followed in their direction)."""

    def __init__(self, lib):
        self.lib = lib

    def _f(self, name, directed):
        return getattr(self.lib, name + ("_directed" if directed else ""))

    def _call(self, name, g, directed, *rest):
        """name's entry point for g: weighted when g carries arc weights
        (g.w, int32 in col order), else the plain or directed form."""
        n, row, col = _csr(g)
        w = getattr(g, "w", None)
        if w is None:
            return self._f(name, directed)(n, _p(row), _p(col), *rest)
        wt = np.ascontiguousarray(w, dtype=np.int32)
        return getattr(self.lib, name + "_weighted")(n, _p(row), _p(col), _p(wt),
                                                     1 if directed else 0, *rest)

    def philox(self, ctr, key):
        c = np.asarray(ctr, dtype=np.uint64)
        k = np.asarray(key, dtype=np.uint64)
        out = np.zeros(4, dtype=np.uint64)
        self.lib.oracle_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
        return out

    def draw_source(self, seed, j, n):
        return int(self.lib.oracle_draw_source(seed, j, n))

    def draw_pair(self, seed, j, n):
        u = ctypes.c_int32()
        v = ctypes.c_int32()
        self.lib.oracle_draw_pair(seed, j, n, ctypes.byref(u), ctypes.byref(v))
        return u.value, v.value

    def brandes(self, g, s, directed=False):
        """-> dist int32[n], sigma (mant f64[n], exp int32[n]), delta f64[n]"""
        n, row, col = _csr(g)
        dist = np.zeros(n, np.int32)
        sm = np.zeros(n, np.float64)
        se = np.zeros(n, np.int32)
        de = np.zeros(n, np.float64)
        _ok(self._call("oracle_brandes", g, directed, int(s), _p(dist), _p(sm), _p(se), _p(de)),
            "oracle_brandes")
        return dist, (sm, se), de

    def bc_exact(self, g, directed=False):
        n, row, col = _csr(g)
        bc = np.zeros(n, np.float64)
        _ok(self._call("oracle_bc_exact", g, directed, _p(bc)), "oracle_bc_exact")
        return bc

    def dependencies(self, g, sources, full=True, total=True, directed=False):
        n, row, col = _csr(g)
        src = np.ascontiguousarray(sources, dtype=np.int32)
        k = src.shape[0]
        f = np.zeros((k, n), np.float64) if full else None
        s = np.zeros(n, np.float64) if total else None
        _ok(self._call("oracle_dependencies", g, directed, _p(src), k, _p(f), _p(s)),
            "oracle_dependencies")
        return f, s

    def pair_dependency(self, g, u, v, directed=False):
        n, row, col = _csr(g)
        y = np.zeros(n, np.float64)
        _ok(self._call("oracle_pair_dependency", g, directed, int(u), int(v), _p(y)),
            "oracle_pair_dependency")
        return y

    def adaptive_source(self, g, targets, c, seed, k_max, directed=False):
        n, row, col = _csr(g)
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = t.shape[0]
        est = np.zeros(T, np.float64)
        k = np.zeros(T, np.int64)
        S = np.zeros(T, np.float64)
        st = np.zeros(T, np.uint8)
        _ok(self._call("oracle_adaptive_source", g, directed, _p(t), T, float(c), int(seed),
                       int(k_max), _p(est), _p(k), _p(S), _p(st)), "oracle_adaptive_source")
        return est, k, S, st

    def adaptive_pair(self, g, targets, rule, eps, c, seed, k_max, directed=False):
        n, row, col = _csr(g)
        t = np.ascontiguousarray(targets, dtype=np.int32)
        T = t.shape[0]
        est = np.zeros(T, np.float64)
        k = np.zeros(T, np.int64)
        S = np.zeros(T, np.float64)
        st = np.zeros(T, np.uint8)
        _ok(self._call("oracle_adaptive_pair", g, directed, _p(t), T, int(rule), float(eps),
                       float(c), int(seed), int(k_max), _p(est), _p(k), _p(S), _p(st)),
            "oracle_adaptive_pair")
        return est, k, S, st

    def source_work(self, g, s):
        n, row, col = _csr(g)
        a = np.zeros(3, np.int64)
        _ok(self.lib.oracle_source_work(n, _p(row), _p(col), int(s), a[0:].ctypes.data,
                                        a[1:].ctypes.data, a[2:].ctypes.data),
            "oracle_source_work")
        return int(a[0]), int(a[1]), int(a[2])

    def pair_work(self, g, u, v):
        n, row, col = _csr(g)
        a = np.zeros(1, np.int64)
        _ok(self.lib.oracle_pair_work(n, _p(row), _p(col), int(u), int(v), _p(a)),
            "oracle_pair_work")
        return int(a[0])

    def bidir_work(self, g, u, v, directed=False):
        """(vertices found, arcs read) by the two-sided search for (u, v)."""
        n, row, col = _csr(g)
        a = np.zeros(2, np.int64)
        _ok(self.lib.oracle_bidir_work(n, _p(row), _p(col), 1 if directed else 0, int(u), int(v),
                                       a[0:].ctypes.data, a[1:].ctypes.data),
            "oracle_bidir_work")
        return int(a[0]), int(a[1])


def sigma_value(mant, exp):
    """Extended path count as a Python float where it fits (else inf)."""
    return np.ldexp(mant, exp)
