"""bcmi: sampled betweenness centrality on an MI355X, Python binding.

Argument marshalling only: every step of the computation runs in the HIP
library libbcmi.so (csrc/), reached through its C ABI (include/bcmi.h).
PyTorch supplies device memory (tensors) and the stream. The binding raises
if the library is missing; there is no fallback path.

Names follow the C ABI: bc_graph_create, bc_exact, bc_dependencies,
bc_pair_dependencies, bc_adaptive_source, bc_adaptive_pair, bc_draw_sources,
bc_draw_pairs. Array arguments are CUDA (HIP) tensors on the graph's device
(or, for a graph set to BC_IO_HOST, contiguous CPU tensors or numpy arrays).
By default the library's device memory comes from torch's caching allocator,
passed in as the ABI's bc_allocator.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libbcmi.so")
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("bcmi.hip", "kernels.hpp", "philox.hpp")]
HEADER = os.path.join(_ROOT, "include", "bcmi.h")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

BC_OK, BC_E_INVALID, BC_E_NOMEM, BC_E_DEVICE, BC_E_UNSUPPORTED = 0, 1, 2, 3, 4
BC_DONE, BC_CAPPED = 0, 1
BC_OUT_FULL, BC_OUT_SUM, BC_OUT_TARGETS = 0, 1, 2
BC_IO_DEVICE, BC_IO_HOST = 0, 1
BC_PAIR_ALG1, BC_PAIR_EPS = 0, 1
BC_SCHED_AUTO, BC_SCHED_BATCHED, BC_SCHED_PER_SOURCE, BC_SCHED_THREADED, BC_SCHED_TUNED = \
    0, 1, 2, 3, 4
BC_SCHED_WORKGROUP = 5
BC_PAIR_SEARCH_AUTO, BC_PAIR_SEARCH_ONE_SIDED, BC_PAIR_SEARCH_BIDIRECTIONAL = 0, 1, 2

EXPORTS = [
    "bc_graph_create", "bc_graph_create_directed", "bc_graph_create_weighted",
    "bc_graph_destroy", "bc_graph_set_stream",
    "bc_graph_set_io",
    "bc_graph_configure", "bc_graph_tune", "bc_graph_plan",
    "bc_graph_info", "bc_exact", "bc_dependencies", "bc_dependencies_noalloc",
    "bc_pair_dependencies",
    "bc_adaptive_source", "bc_adaptive_pair", "bc_draw_sources", "bc_draw_pairs",
    "bc_last_stats", "bc_last_error", "bc_profile_enable", "bc_profile_read",
    "bc_server_create", "bc_server_destroy", "bc_server_add_graph", "bc_server_submit",
    "bc_server_step", "bc_server_set_lanes", "bc_server_poll", "bc_server_now", "bc_server_stats_get",
    "bc_server_graph_width",
]
BC_QUERY_SOURCE, BC_QUERY_PAIR = 0, 1


def build(force: bool = True) -> str:
    """Compile csrc/bcmi.hip for gfx950 into libbcmi.so (hipcc)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-I" + os.path.join(_ROOT, "include"),
                                     os.path.join(_HERE, "csrc", "bcmi.hip"), "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class BcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("bcmi status %d: %s" % (status, msg))
        self.status = status


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row", ctypes.c_void_p),
                ("row_is_i64", ctypes.c_int32), ("col", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("bottom_up", ctypes.c_double), ("split_entries", ctypes.c_int64),
                ("level_loop", ctypes.c_int32), ("sampler_batch", ctypes.c_int32),
                ("pair_search", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("samples_executed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("levels", ctypes.c_int64), ("extended", ctypes.c_int32),
                ("batch_width", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("pair_search", ctypes.c_int32), ("bottom_up", ctypes.c_double)]


class _KProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("units_a", ctypes.c_int64),
                ("units_b", ctypes.c_int64), ("algo_bytes", ctypes.c_double)]


class _Query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("target", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("c", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("k_max", ctypes.c_int64),
                ("arrival_s", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("graph", ctypes.c_int32), ("status", ctypes.c_int32),
                ("est", ctypes.c_double), ("samples", ctypes.c_int64), ("S", ctypes.c_double),
                ("arrival_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("queued", "active", "finished", "rounds",
                                               "samples_executed", "samples_used",
                                               "resident_bytes", "workspace_bytes",
                                               "budget_bytes", "split_rounds")]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


def _torch_alloc(size, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(size), torch.cuda.current_device(),
                                                  torch.cuda.current_stream())
    except Exception:       # out of memory: the library reports BC_E_NOMEM
        return None


def _torch_free(ptr, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(ptr)
    except Exception:
        pass


# torch's caching allocator as a bc_allocator (kept alive for the process)
TORCH_ALLOCATOR = _Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


def _allocator(which):
    """'torch' -> torch's caching allocator, 'hip' -> the library's hipMalloc."""
    if which == "torch":
        return ctypes.byref(TORCH_ALLOCATOR)
    if which == "hip":
        return None
    raise ValueError("allocator must be 'torch' or 'hip'")


def _csr_arrays(row, col):
    """Host CSR arrays: int64 or int32 row offsets (kept as given), int32 columns."""
    import numpy as np
    row = np.asarray(row)
    row = np.ascontiguousarray(row, dtype=np.int32 if row.dtype == np.int32 else np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    csr = _Csr(row.shape[0] - 1, col.shape[0], row.ctypes.data, 1 if row.dtype == np.int64 else 0,
               col.ctypes.data if col.shape[0] else None)
    return csr, (row, col)


_lib = None


def load_library(path: str | None = None):
    """Load libbcmi.so; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    # torch ships its own HIP runtime under the same soname as ROCm's; loading
    # torch first makes this library bind to that one runtime in the process
    import torch  # noqa: F401
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libbcmi.so is not built (%s); run __graft_entry__.build()" % p)
    lib = ctypes.CDLL(p)
    c = ctypes
    V = c.c_void_p
    lib.bc_last_error.restype = c.c_char_p
    lib.bc_last_error.argtypes = []
    lib.bc_graph_destroy.restype = None
    lib.bc_graph_destroy.argtypes = [V]
    lib.bc_server_destroy.restype = None
    lib.bc_server_destroy.argtypes = [V]
    sigs = {
        "bc_graph_create": [c.POINTER(_Csr), V, V, c.POINTER(V)],
        "bc_graph_create_directed": [c.POINTER(_Csr), V, V, c.POINTER(V)],
        "bc_graph_create_weighted": [c.POINTER(_Csr), V, c.c_int32, V, V, c.POINTER(V)],
        "bc_graph_set_stream": [V, V],
        "bc_graph_set_io": [V, c.c_int32],
        "bc_graph_configure": [V, c.POINTER(_Config)],
        "bc_graph_tune": [V, c.POINTER(_Config)],
        "bc_graph_plan": [V, c.POINTER(_Config)],
        "bc_graph_info": [V, c.POINTER(c.c_int64), c.POINTER(c.c_int64)],
        "bc_exact": [V, V],
        "bc_dependencies": [V, V, c.c_int64, c.c_int32, V, V, V, V, V, c.c_int32],
        "bc_pair_dependencies": [V, V, V, c.c_int64, V],
        "bc_dependencies_noalloc": [V, V, c.c_int64, c.c_int32, V],
        "bc_adaptive_source": [V, V, c.c_int32, c.c_double, c.c_uint64, c.c_int64, V, V, V, V],
        "bc_adaptive_pair": [V, V, c.c_int32, c.c_int32, c.c_double, c.c_double, c.c_uint64,
                             c.c_int64, V, V, V, V],
        "bc_draw_sources": [V, c.c_uint64, c.c_int64, c.c_int64, V],
        "bc_draw_pairs": [V, c.c_uint64, c.c_int64, c.c_int64, V, V],
        "bc_last_stats": [V, c.POINTER(_Stats)],
        "bc_profile_enable": [V, c.c_int32],
        "bc_server_create": [c.c_size_t, c.c_int32, V, V, c.POINTER(V)],
        "bc_server_graph_width": [V, c.c_int32, c.POINTER(c.c_int32), c.POINTER(c.c_int32)],
        "bc_server_add_graph": [V, c.POINTER(_Csr), c.POINTER(c.c_int32)],
        "bc_server_submit": [V, c.POINTER(_Query), c.POINTER(c.c_int64)],
        "bc_server_step": [V, c.POINTER(c.c_int32)],
        "bc_server_set_lanes": [V, c.c_int32],
        "bc_server_poll": [V, c.POINTER(_Result), c.c_int32, c.POINTER(c.c_int32)],
        "bc_server_now": [V, c.POINTER(c.c_double)],
        "bc_server_stats_get": [V, c.POINTER(_ServerStats)],
        "bc_profile_read": [V, c.POINTER(_KProf), c.c_int32, c.POINTER(c.c_int32)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.restype = c.c_int
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(rc):
    if rc != BC_OK:
        raise BcError(rc, _lib.bc_last_error().decode())


def _ptr(t, dtype=None, numel=None, name="tensor", host=False):
    """Pointer of a contiguous tensor (None -> NULL): a device tensor, or with
    host=True a CPU tensor or numpy array (graphs set to BC_IO_HOST)."""
    if t is None:
        return None
    import numpy as np
    import torch
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(t)
    if host:
        if t.is_cuda:
            raise ValueError("%s must be a host array (the graph is set to BC_IO_HOST)" % name)
    elif not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    return t.data_ptr()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Graph:
    """Handle to a device-resident CSR graph (bc_graph). row may be int64 or
    int32 offsets; allocator 'torch' (default) or 'hip'; directed=True reads
    row/col as out-neighbour lists (bc_graph_create_directed); weights (int32
    per arc of col, positive) make it a weighted graph (bc_graph_create_weighted)."""

    def __init__(self, row, col, allocator="torch", directed=False, weights=None):
        lib = load_library()
        csr, keep = _csr_arrays(row, col)
        h = ctypes.c_void_p()
        self._h = None
        if weights is not None:
            import numpy as np
            wt = np.ascontiguousarray(np.asarray(weights), dtype=np.int32)
            if wt.shape != (int(csr.nnz),):
                raise ValueError("weights need one entry per arc")
            _check(lib.bc_graph_create_weighted(ctypes.byref(csr), wt.ctypes.data,
                                                1 if directed else 0, _allocator(allocator),
                                                _stream(), ctypes.byref(h)))
        else:
            create = lib.bc_graph_create_directed if directed else lib.bc_graph_create
            _check(create(ctypes.byref(csr), _allocator(allocator), _stream(), ctypes.byref(h)))
        self.weighted = weights is not None
        self.directed = bool(directed)
        self._h = h
        self.n = int(csr.n)
        self.nnz = int(csr.nnz)
        self.host_io = False
        del keep

    def set_io(self, host: bool):
        """BC_IO_HOST: later compute calls take host arrays."""
        _check(_lib.bc_graph_set_io(self.handle, BC_IO_HOST if host else BC_IO_DEVICE))
        self.host_io = bool(host)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph is closed")
        _check(_lib.bc_graph_set_stream(self._h, _stream()))
        return self._h

    def configure(self, schedule=BC_SCHED_AUTO, batch=0, bottom_up=0.0, split_entries=0,
                  level_loop=0, sampler_batch=0, pair_search=0):
        cfg = _Config(int(schedule), int(batch), float(bottom_up), int(split_entries),
                      int(level_loop), int(sampler_batch), int(pair_search))
        _check(_lib.bc_graph_configure(self.handle, ctypes.byref(cfg)))

    def tune(self):
        """Time candidate plans, install the fastest and return it (a dict)."""
        cfg = _Config()
        _check(_lib.bc_graph_tune(self.handle, ctypes.byref(cfg)))
        return {f: getattr(cfg, f) for f, _ in _Config._fields_}

    def plan(self):
        """The plan compute calls use now (a dict)."""
        cfg = _Config()
        _check(_lib.bc_graph_plan(self.handle, ctypes.byref(cfg)))
        return {f: getattr(cfg, f) for f, _ in _Config._fields_}

    def stats(self):
        st = _Stats()
        _check(_lib.bc_last_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _Stats._fields_}

    def profile(self, enable: bool):
        _check(_lib.bc_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self):
        arr = (_KProf * 16)()
        cnt = ctypes.c_int32()
        _check(_lib.bc_profile_read(self.handle, arr, 16, ctypes.byref(cnt)))
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
                 "units_a": arr[i].units_a, "units_b": arr[i].units_b,
                 "algo_bytes": arr[i].algo_bytes} for i in range(cnt.value)]

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.bc_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Query server with continuous batching over device-resident graphs."""

    def __init__(self, hbm_budget_bytes, max_batch=256, allocator="torch"):
        lib = load_library()
        h = ctypes.c_void_p()
        self._h = None
        _check(lib.bc_server_create(int(hbm_budget_bytes), int(max_batch), _allocator(allocator),
                                    _stream(), ctypes.byref(h)))
        self._h = h

    def add_graph(self, row, col) -> int:
        csr, keep = _csr_arrays(row, col)
        gid = ctypes.c_int32()
        _check(_lib.bc_server_add_graph(self._h, ctypes.byref(csr), ctypes.byref(gid)))
        del keep
        return gid.value

    def graph_width(self, graph):
        w = ctypes.c_int32()
        sch = ctypes.c_int32()
        _check(_lib.bc_server_graph_width(self._h, int(graph), ctypes.byref(w), ctypes.byref(sch)))
        return w.value, sch.value

    def submit(self, graph, target, kind, seed, k_max, c=1.0, eps=0.1, rule=BC_PAIR_EPS,
               arrival_s=-1.0) -> int:
        q = _Query(int(graph), int(target), int(kind), int(rule), float(c), float(eps),
                   int(seed), int(k_max), float(arrival_s))
        qid = ctypes.c_int64()
        _check(_lib.bc_server_submit(self._h, ctypes.byref(q), ctypes.byref(qid)))
        return qid.value

    def set_lanes(self, lanes: int):
        """Rounds of up to `lanes` graphs at once, each on its own stream."""
        _check(_lib.bc_server_set_lanes(self._h, int(lanes)))

    def step(self) -> int:
        done = ctypes.c_int32()
        _check(_lib.bc_server_step(self._h, ctypes.byref(done)))
        return done.value

    def poll(self, max_results=4096):
        arr = (_Result * max_results)()
        cnt = ctypes.c_int32()
        _check(_lib.bc_server_poll(self._h, arr, max_results, ctypes.byref(cnt)))
        return [{f: getattr(arr[i], f) for f, _ in _Result._fields_} for i in range(cnt.value)]

    def now(self) -> float:
        t = ctypes.c_double()
        _check(_lib.bc_server_now(self._h, ctypes.byref(t)))
        return t.value

    def stats(self):
        st = _ServerStats()
        _check(_lib.bc_server_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.bc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bc_graph_create(row, col) -> Graph:
    return Graph(row, col)


def _numel(t):
    return int(t.numel()) if hasattr(t, "numel") else int(t.size)


def bc_exact(g: Graph, out):
    import torch
    _check(_lib.bc_exact(g.handle, _ptr(out, torch.float64, g.n, "out", g.host_io)))


def bc_dependencies(g: Graph, sources, out_mode, out, dist_out=None, sigma_mant=None,
                    sigma_exp=None, targets=None):
    import torch
    h = g.host_io
    k = _numel(sources)
    T = _numel(targets) if targets is not None else 0
    need = {BC_OUT_FULL: k * g.n, BC_OUT_SUM: g.n, BC_OUT_TARGETS: k * T}[int(out_mode)]
    _check(_lib.bc_dependencies(
        g.handle, _ptr(sources, torch.int32, k, "sources", h), k, int(out_mode),
        _ptr(out, torch.float64, need, "out", h),
        _ptr(dist_out, torch.int32, k * g.n, "dist_out", h),
        _ptr(sigma_mant, torch.float64, k * g.n, "sigma_mant", h),
        _ptr(sigma_exp, torch.int32, k * g.n, "sigma_exp", h),
        _ptr(targets, torch.int32, T, "targets", h), T))


def bc_dependencies_noalloc(g: Graph, sources, out_mode, out):
    """bc_dependencies (BC_OUT_FULL / BC_OUT_SUM) with no device allocation:
    the library's fixed scratch array holds the engine's buffers."""
    import torch
    k = _numel(sources)
    need = k * g.n if int(out_mode) == BC_OUT_FULL else g.n
    _check(_lib.bc_dependencies_noalloc(g.handle, _ptr(sources, torch.int32, k, "sources"), k,
                                        int(out_mode), _ptr(out, torch.float64, need, "out")))


def bc_pair_dependencies(g: Graph, us, vs, out):
    import torch
    h = g.host_io
    k = _numel(us)
    if _numel(vs) != k:
        raise ValueError("us and vs differ in length")
    _check(_lib.bc_pair_dependencies(g.handle, _ptr(us, torch.int32, k, "us", h),
                                     _ptr(vs, torch.int32, k, "vs", h), k,
                                     _ptr(out, torch.float64, k * g.n, "out", h)))


def bc_adaptive_source(g: Graph, targets, c, seed, k_max, out_est, out_samples, out_S,
                       out_status):
    import torch
    h = g.host_io
    T = _numel(targets)
    _check(_lib.bc_adaptive_source(
        g.handle, _ptr(targets, torch.int32, T, "targets", h), T, float(c), int(seed), int(k_max),
        _ptr(out_est, torch.float64, T, "out_est", h),
        _ptr(out_samples, torch.int64, T, "out_samples", h),
        _ptr(out_S, torch.float64, T, "out_S", h), _ptr(out_status, torch.uint8, T, "out_status", h)))


def bc_adaptive_pair(g: Graph, targets, rule, eps, c, seed, k_max, out_est, out_samples, out_S,
                     out_status):
    import torch
    h = g.host_io
    T = _numel(targets)
    _check(_lib.bc_adaptive_pair(
        g.handle, _ptr(targets, torch.int32, T, "targets", h), T, int(rule), float(eps), float(c),
        int(seed), int(k_max), _ptr(out_est, torch.float64, T, "out_est", h),
        _ptr(out_samples, torch.int64, T, "out_samples", h),
        _ptr(out_S, torch.float64, T, "out_S", h),
        _ptr(out_status, torch.uint8, T, "out_status", h)))


def bc_draw_sources(g: Graph, seed, j0, count, out_u):
    import torch
    _check(_lib.bc_draw_sources(g.handle, int(seed), int(j0), int(count),
                                _ptr(out_u, torch.int32, count, "out_u", g.host_io)))


def bc_draw_pairs(g: Graph, seed, j0, count, out_u, out_v):
    import torch
    h = g.host_io
    _check(_lib.bc_draw_pairs(g.handle, int(seed), int(j0), int(count),
                              _ptr(out_u, torch.int32, count, "out_u", h),
                              _ptr(out_v, torch.int32, count, "out_v", h)))


# ---------------------------------------------------- allocating conveniences

def _dev():
    import torch
    return torch.device("cuda", torch.cuda.current_device())


def exact(g: Graph):
    import torch
    out = torch.empty(g.n, dtype=torch.float64, device=_dev())
    bc_exact(g, out)
    return out


def dependencies(g: Graph, sources, mode=BC_OUT_FULL, dist=False, sigma=False):
    import torch
    k = sources.numel()
    out = torch.empty(k * g.n if mode == BC_OUT_FULL else g.n, dtype=torch.float64, device=_dev())
    d = torch.empty(k * g.n, dtype=torch.int32, device=_dev()) if dist else None
    sm = torch.empty(k * g.n, dtype=torch.float64, device=_dev()) if sigma else None
    se = torch.empty(k * g.n, dtype=torch.int32, device=_dev()) if sigma else None
    bc_dependencies(g, sources, mode, out, d, sm, se)
    if mode == BC_OUT_FULL:
        out = out.view(k, g.n)
    return out, (d.view(k, g.n) if dist else None), \
        ((sm.view(k, g.n), se.view(k, g.n)) if sigma else None)


def target_dependencies(g: Graph, sources, targets):
    """delta_{sources[i].}(targets[t]) as a k x T tensor (BC_OUT_TARGETS)."""
    import torch
    k, T = sources.numel(), targets.numel()
    out = torch.empty(k * T, dtype=torch.float64, device=_dev())
    bc_dependencies(g, sources, BC_OUT_TARGETS, out, targets=targets)
    return out.view(k, T)


def pair_dependencies(g: Graph, us, vs):
    import torch
    out = torch.empty(us.numel() * g.n, dtype=torch.float64, device=_dev())
    bc_pair_dependencies(g, us, vs, out)
    return out.view(us.numel(), g.n)


def _sampler_outputs(T):
    import torch
    d = _dev()
    return (torch.empty(T, dtype=torch.float64, device=d), torch.empty(T, dtype=torch.int64, device=d),
            torch.empty(T, dtype=torch.float64, device=d), torch.empty(T, dtype=torch.uint8, device=d))


def adaptive_source(g: Graph, targets, c, seed, k_max):
    est, k, S, st = _sampler_outputs(targets.numel())
    bc_adaptive_source(g, targets, c, seed, k_max, est, k, S, st)
    return est, k, S, st


def adaptive_pair(g: Graph, targets, rule, eps, c, seed, k_max):
    est, k, S, st = _sampler_outputs(targets.numel())
    bc_adaptive_pair(g, targets, rule, eps, c, seed, k_max, est, k, S, st)
    return est, k, S, st
