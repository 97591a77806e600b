"""Seeded synthetic inputs: graphs, source lists and target lists.

Input generation only. Nothing here computes distances, path counts,
dependencies or estimates; both the CPU oracle and the GPU library consume the
CSR arrays built here byte for byte.

CSR convention used everywhere in this repository:
  row: int64[n+1] offsets, col: int32[nnz] neighbour ids,
  symmetric (undirected), rows sorted ascending, no self-loops, no duplicates.

Random streams: numpy's Philox4x64-10 bit generator keyed (seed, stream) with
stream ids graph=2, sources=0, pairs=1, arrivals=3; the Barabasi-Albert
generator runs in C (gen.c) with a SplitMix64 stream seeded from the same key.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

STREAM_SOURCES = 0
STREAM_PAIRS = 1
STREAM_GRAPH = 2
STREAM_ARRIVALS = 3


def build_native(force: bool = False) -> str:
    """Compile gen.c into libgraphgen.so (gcc, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-shared", "-fPIC", "-std=c11",
                               os.path.join(_HERE, "gen.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _native():
    global _lib
    if _lib is None:
        build_native()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.graphgen_ba.restype = ctypes.c_int64
        lib.graphgen_ba.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_void_p, ctypes.c_void_p]
        lib.graphgen_rmat.restype = ctypes.c_int64
        lib.graphgen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_void_p]
        lib.graphgen_csr.restype = ctypes.c_int64
        lib.graphgen_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class CSR:
    n: int
    row: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    name: str = ""
    directed: bool = False   # row v lists v's out-neighbours (arcs v -> w)
    w: np.ndarray | None = None   # int32[nnz] arc weights (col order), or None

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m_undirected(self) -> int:
        return self.nnz // 2

    def degree(self) -> np.ndarray:
        return np.diff(self.row)

    def neighbours(self, v: int) -> np.ndarray:
        return self.col[self.row[v]:self.row[v + 1]]


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


def from_edges(n: int, src, dst, name: str = "") -> CSR:
    """Symmetric, sorted, deduplicated CSR from an undirected edge list."""
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    dst = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    assert src.shape == dst.shape
    if n <= 0:
        raise ValueError("n must be positive")
    row = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(1, 2 * src.shape[0]), dtype=np.int32)
    nnz = _native().graphgen_csr(n, src.shape[0], src.ctypes.data, dst.ctypes.data,
                                 row.ctypes.data, col.ctypes.data)
    if nnz < 0:
        raise ValueError("edge list has an endpoint outside [0, n)")
    return CSR(n, row, col[:nnz].copy(), name)


def from_arcs(n: int, src, dst, name: str = "") -> CSR:
    """Directed CSR of out-neighbours from an arc list: rows sorted ascending,
    self-loops and repeated arcs dropped."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    assert src.shape == dst.shape
    if n <= 0:
        raise ValueError("n must be positive")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("arc list has an endpoint outside [0, n)")
    keep = src != dst
    key = np.unique(src[keep] * n + dst[keep])
    a, b = key // n, key % n
    row = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row, a + 1, 1)
    row = np.cumsum(row)
    return CSR(n, row, b.astype(np.int32), name, directed=True)


def directed_path(n: int) -> CSR:
    return from_arcs(n, np.arange(n - 1), np.arange(1, n), "dpath%d" % n)


def directed_cycle(n: int) -> CSR:
    return from_arcs(n, np.arange(n), (np.arange(n) + 1) % n, "dcycle%d" % n)


def out_star(n: int) -> CSR:
    """Vertex 0 with an arc to every other vertex."""
    return from_arcs(n, np.zeros(n - 1, np.int64), np.arange(1, n), "ostar%d" % n)


def bidirected(g: CSR) -> CSR:
    """An undirected CSR read as a directed one (every edge an arc both ways)."""
    return CSR(g.n, g.row, g.col, g.name + "_bidir", directed=True)


def rmat_directed(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> CSR:
    """The R-MAT draws of rmat() kept as arcs (not symmetrised)."""
    n = 1 << scale
    ne = edge_factor * n
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    key = (int(seed) * 0x100000001B3 + STREAM_GRAPH) & ((1 << 64) - 1)
    got = _native().graphgen_rmat(scale, edge_factor, a, b, c, key, src.ctypes.data,
                                  dst.ctypes.data)
    if got != ne:
        raise RuntimeError("graphgen_rmat failed")
    return from_arcs(n, src, dst, "drmat%d_%d" % (scale, edge_factor))


def with_weights(g: CSR, wmax: int, seed: int, stream: int = 7) -> CSR:
    """g with positive integer arc weights drawn uniformly from [1, wmax]
    (Philox key (seed, stream)). Undirected graphs draw one weight per edge,
    so both arcs of an edge carry it; directed graphs one per arc."""
    r = rng(seed, stream)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row))
    dst = g.col.astype(np.int64)
    if g.directed:
        w = r.integers(1, wmax + 1, g.nnz)
    else:
        # weight of edge {a, b}: a draw indexed by the edge's rank among the
        # arcs a -> b with a < b (the same rank from either end)
        lo, hi = np.minimum(src, dst), np.maximum(src, dst)
        key = lo * g.n + hi
        uniq, inv = np.unique(key, return_inverse=True)
        w = r.integers(1, wmax + 1, uniq.shape[0])[inv]
    return CSR(g.n, g.row, g.col, g.name + "-w%d" % wmax, g.directed, w.astype(np.int32))


def relabel_subgraph(g: CSR, keep: np.ndarray, name: str = "") -> CSR:
    """Induced subgraph on the vertices where keep is True, ids renumbered in order."""
    newid = -np.ones(g.n, dtype=np.int64)
    idx = np.nonzero(keep)[0]
    newid[idx] = np.arange(idx.shape[0])
    src = np.repeat(np.arange(g.n), np.diff(g.row))
    dst = g.col.astype(np.int64)
    m = keep[src] & keep[dst] & (src < dst)
    return from_edges(int(idx.shape[0]), newid[src[m]], newid[dst[m]], name)


def largest_component(g: CSR) -> CSR:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row), shape=(g.n, g.n))
    ncomp, lab = connected_components(a, directed=False)
    if ncomp == 1:
        return g
    big = np.argmax(np.bincount(lab))
    return relabel_subgraph(g, lab == big, g.name + "-lcc")


# ----------------------------------------------------------------- families

def path(n: int) -> CSR:
    a = np.arange(n - 1)
    return from_edges(n, a, a + 1, "path%d" % n)


def star(n: int) -> CSR:
    """Vertex 0 is the centre; leaves 1..n-1."""
    a = np.arange(1, n)
    return from_edges(n, np.zeros_like(a), a, "star%d" % n)


def cycle(n: int) -> CSR:
    a = np.arange(n)
    return from_edges(n, a, (a + 1) % n, "cycle%d" % n)


def complete(n: int) -> CSR:
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j, "K%d" % n)


def complete_bipartite(a: int, b: int) -> CSR:
    """Part A = 0..a-1, part B = a..a+b-1."""
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, i.ravel(), j.ravel(), "K%d,%d" % (a, b))


def grid(x: int, y: int) -> CSR:
    """x-by-y 4-neighbour grid; vertex (i, j) has id i*y + j."""
    ids = np.arange(x * y).reshape(x, y)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(x * y, s, d, "grid%dx%d" % (x, y))


def er(n: int, p: float, seed: int) -> CSR:
    """G(n, p): each unordered pair independently with probability p."""
    r = rng(seed, STREAM_GRAPH)
    i, j = np.triu_indices(n, 1)
    keep = r.random(i.shape[0]) < p
    return from_edges(n, i[keep], j[keep], "er%d" % n)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int) -> CSR:
    """R-MAT (Chakrabarti et al. 2004): edge_factor * 2^scale generated edges,
    quadrant probabilities a, b, c, d = 1-a-b-c at every bit, no noise, no
    relabelling; symmetrised, self-loops and duplicates dropped, isolated
    vertices kept (n = 2^scale). Drawn in C from a SplitMix64 stream keyed by
    (seed, graph stream)."""
    n = 1 << scale
    ne = edge_factor * n
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    key = (int(seed) * 0x100000001B3 + STREAM_GRAPH) & ((1 << 64) - 1)
    got = _native().graphgen_rmat(scale, edge_factor, a, b, c, key, src.ctypes.data,
                                  dst.ctypes.data)
    if got != ne:
        raise RuntimeError("graphgen_rmat failed")
    return from_edges(n, src, dst, "rmat%d_%d" % (scale, edge_factor))


def ba(n: int, m: int, seed: int) -> CSR:
    """Barabasi-Albert: K_{m+1} seed clique, then m degree-proportional distinct
    targets per new vertex; m(m+1)/2 + m(n-m-1) undirected edges."""
    ne = m * (m + 1) // 2 + m * (n - m - 1)
    src = np.zeros(ne, dtype=np.int32)
    dst = np.zeros(ne, dtype=np.int32)
    key = (int(seed) * 0x100000001B3 + STREAM_GRAPH) & ((1 << 64) - 1)
    got = _native().graphgen_ba(n, m, key, src.ctypes.data, dst.ctypes.data)
    if got != ne:
        raise RuntimeError("graphgen_ba failed")
    return from_edges(n, src, dst, "ba%d_%d" % (n, m))


def powerlaw_cluster(n: int, m: int, p: float, seed: int) -> CSR:
    """Holme-Kim growth: preferential attachment with triad formation. Each new
    vertex makes m edges; the first goes to a degree-proportional target, and
    each later one, with probability p, to a random neighbour of the previous
    target that is not yet linked (a triangle), else to another
    degree-proportional target. Starts from the clique K_{m+1}."""
    r = rng(seed, STREAM_GRAPH)
    adj = [set() for _ in range(n)]
    ends = []                       # every edge endpoint: degree-proportional draws
    src, dst = [], []

    def link(a, b):
        adj[a].add(b)
        adj[b].add(a)
        ends.extend((a, b))
        src.append(a)
        dst.append(b)

    for a in range(m + 1):
        for b in range(a + 1, m + 1):
            link(a, b)
    for v in range(m + 1, n):
        made = 0
        last = -1
        while made < m:
            u = -1
            if last >= 0 and made > 0 and r.random() < p:
                cand = [w for w in adj[last] if w != v and w not in adj[v]]
                if cand:
                    u = cand[int(r.integers(len(cand)))]
            if u < 0:
                while True:
                    u = ends[int(r.integers(len(ends)))]
                    if u != v and u not in adj[v]:
                        break
            link(v, u)
            last = u
            made += 1
    return from_edges(n, np.array(src), np.array(dst), "plc%d_%d" % (n, m))


def small_world(n: int, k: int, p: float, seed: int) -> CSR:
    """Watts-Strogatz: the ring lattice where each vertex links to its k/2
    nearest vertices on either side, then each lattice edge (i, i+j), taken in
    order of j and then i, moves its far end with probability p to a uniform
    vertex that is neither i nor already linked to it."""
    r = rng(seed, STREAM_GRAPH)
    adj = [set() for _ in range(n)]
    for i in range(n):
        for j in range(1, k // 2 + 1):
            b = (i + j) % n
            adj[i].add(b)
            adj[b].add(i)
    for j in range(1, k // 2 + 1):
        for i in range(n):
            b = (i + j) % n
            if b not in adj[i] or r.random() >= p or len(adj[i]) >= n - 1:
                continue
            while True:
                w = int(r.integers(n))
                if w != i and w not in adj[i]:
                    break
            adj[i].discard(b)
            adj[b].discard(i)
            adj[i].add(w)
            adj[w].add(i)
    src = [a for a in range(n) for b in adj[a] if a < b]
    dst = [b for a in range(n) for b in adj[a] if a < b]
    return from_edges(n, np.array(src), np.array(dst), "ws%d_%d" % (n, k))


def average_clustering(g: CSR) -> float:
    """Mean over vertices of the local clustering coefficient (0 below degree 2)."""
    import scipy.sparse as sp
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.float64), g.col, g.row), shape=(g.n, g.n))
    tri = np.asarray((a @ a).multiply(a).sum(axis=1)).ravel() / 2.0
    d = np.diff(g.row).astype(np.float64)
    pairs = d * (d - 1) / 2.0
    c = np.divide(tri, pairs, out=np.zeros_like(tri), where=pairs > 0)
    return float(c.mean())


def grid_percolated(side: int, frac: float, seed: int) -> CSR:
    """side x side 4-neighbour grid with floor(frac*E) edges deleted uniformly
    without replacement, reduced to its largest connected component."""
    r = rng(seed, STREAM_GRAPH)
    ids = np.arange(side * side, dtype=np.int64).reshape(side, side)
    s = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    d = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    ne = s.shape[0]
    ndel = int(np.floor(frac * ne))
    drop = r.choice(ne, size=ndel, replace=False)
    keep = np.ones(ne, dtype=bool)
    keep[drop] = False
    g = from_edges(side * side, s[keep], d[keep], "grid%d_p%g" % (side, frac))
    return largest_component(g)


# ----------------------------------------------------------------- samples

def philox_sources(seed: int, count: int, n: int, stream: int = STREAM_SOURCES) -> np.ndarray:
    """Sources for a fixed-list run: word 0 of Philox4x64-10 block j (key
    (seed, stream)) mapped to floor(w * n / 2^64), j = 0..count-1.

    numpy's Philox emits block c+1 first when its counter is c, so the counter
    starts at 2^256 - 1 (which wraps to block 0)."""
    ones = np.full(4, np.iinfo(np.uint64).max, dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64), counter=ones)
    raw = bg.random_raw(4 * count).reshape(count, 4)[:, 0]
    hi = [(int(w) * n) >> 64 for w in raw]
    return np.asarray(hi, dtype=np.int32)


def top_degree(g: CSR, k: int) -> np.ndarray:
    """k highest-degree vertices, ties broken by lower id."""
    deg = g.degree()
    order = np.lexsort((np.arange(g.n), -deg))
    return order[:k].astype(np.int32)


def degree_percentile_targets(g: CSR, k: int, min_degree: int = 2) -> np.ndarray:
    """Vertices at degree percentiles (j + 1/2)/k, j = 0..k-1, among the
    vertices of degree >= min_degree sorted by (degree, id)."""
    deg = g.degree()
    cand = np.nonzero(deg >= min_degree)[0]
    order = cand[np.lexsort((cand, deg[cand]))]
    pos = ((np.arange(k) + 0.5) / k * order.shape[0]).astype(np.int64)
    return order[np.minimum(pos, order.shape[0] - 1)].astype(np.int32)


def serving_graph_params(seed: int):
    """Scale in 10..18 and edge factor in 8..32, each uniform, from the graph's seed."""
    r = rng(seed, 4)
    scale = int(10 + np.floor(r.random() * 9))
    ef = int(8 + np.floor(r.random() * 25))
    return scale, ef


def serving_graphs(count: int = 200, first_seed: int = 100, threads: int = 8):
    """R-MAT graphs with seeds first_seed.. (parameters from serving_graph_params),
    built on a thread pool (the C generators run without the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(i):
        seed = first_seed + i
        scale, ef = serving_graph_params(seed)
        return rmat(scale, ef, 0.57, 0.19, 0.19, seed=seed)

    _native()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(count)))


def serving_queries(graphs, count: int, rate_qps: float, seed: int = 3):
    """Poisson arrivals at rate_qps; graph uniform; target degree-weighted;
    half source queries (c in {2, 5, 10}, k_max 1024), half pair queries
    (eps in {0.05, 0.1}, k_max 65536); query seed = query id."""
    r = rng(seed, STREAM_ARRIVALS)
    t = np.cumsum(r.exponential(1.0 / rate_qps, count))
    out = []
    for i in range(count):
        gi = int(r.integers(0, len(graphs)))
        deg = graphs[gi].degree().astype(np.float64)
        target = int(np.searchsorted(np.cumsum(deg), r.random() * deg.sum(), side="right"))
        target = min(target, graphs[gi].n - 1)
        if r.random() < 0.5:
            out.append(dict(arrival=float(t[i]), graph=gi, target=target, kind=0,
                            c=float(r.choice([2.0, 5.0, 10.0])), eps=0.1, seed=i, k_max=1024))
        else:
            out.append(dict(arrival=float(t[i]), graph=gi, target=target, kind=1, c=1.0,
                            eps=float(r.choice([0.05, 0.1])), seed=i, k_max=65536))
    return out


# ----------------------------------------------------------------- configs

def config_graph(name: str) -> CSR:
    """The synthetic workloads, by name (sizes in the docstrings above)."""
    if name == "er2000":
        return er(2000, 8.0 / 1999.0, seed=1)
    if name == "rmat16":
        return rmat(16, 16, 0.57, 0.19, 0.19, seed=2)
    if name == "ba1m":
        return ba(1 << 20, 5, seed=7)
    if name == "grid2048":
        return grid_percolated(2048, 0.05, seed=3)
    raise KeyError(name)
