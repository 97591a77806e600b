"""The C ABI's memory and output conventions, on the GPU:
  - the caller's bc_allocator (here torch's caching allocator) supplies every
    device byte of a handle; the hipMalloc default gives the same results;
  - BC_OUT_TARGETS equals the BC_OUT_FULL columns of the targets, bit for bit;
  - BC_IO_HOST takes host arrays and returns the device-mode results;
  - int32 row offsets (row_is_i64 = 0) give the int64-offset results.
Each case prints its name before it touches the GPU.
"""
import ctypes
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


def test_torch_allocator_supplies_the_workspace(dev):
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    src = gg.philox_sources(3, 600, g.n)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    say("allocator torch")
    G = bc.Graph(g.row, g.col, allocator="torch")
    csr = torch.cuda.memory_allocated() - base
    assert csr >= 8 * (g.n + 1) + 4 * g.nnz          # the graph's device copy
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    before = torch.cuda.memory_allocated()
    bc.bc_dependencies(G, T(src, dev), bc.BC_OUT_SUM, out)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated() - before
    # the batch's value pool alone is 8 bytes per (vertex, source)
    assert grown >= 8 * g.n * G.stats()["batch_width"], grown
    G.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before - csr
    say("allocator hip")
    H = bc.Graph(g.row, g.col, allocator="hip")
    mid = torch.cuda.memory_allocated()
    out2 = torch.empty(g.n, dtype=torch.float64, device=dev)
    bc.bc_dependencies(H, T(src, dev), bc.BC_OUT_SUM, out2)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == mid + out2.numel() * 8   # nothing from torch
    H.close()
    assert torch.equal(out, out2)
    _, want = O.dependencies(g, src, full=False, total=True)
    assert_close(out.cpu().numpy(), want, what="allocator sum")


@pytest.mark.parametrize("sched", [bc.BC_SCHED_BATCHED, bc.BC_SCHED_THREADED,
                                   bc.BC_SCHED_PER_SOURCE], ids=["wave", "pair", "per-source"])
def test_targets_mode_equals_full_columns(dev, sched):
    g = gg.rmat(11, 8, 0.57, 0.19, 0.19, seed=1)
    G = bc.Graph(g.row, g.col)
    G.configure(sched, 128 if sched != bc.BC_SCHED_PER_SOURCE else 0, 0.0)
    k = 40 if sched == bc.BC_SCHED_PER_SOURCE else 300
    src = gg.philox_sources(8, k, g.n)
    tg = np.concatenate([gg.top_degree(g, 5), [src[0], src[1], 0, g.n - 1]]).astype(np.int32)
    say("targets mode sched", sched)
    full, _, _ = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL)
    got = bc.target_dependencies(G, T(src, dev), T(tg, dev))
    assert got.shape == (k, tg.size)
    assert torch.equal(got, full[:, T(tg.astype(np.int64), dev)])
    for i in (0, 1, k - 1):
        _, _, de = O.brandes(g, int(src[i]))
        assert_close(got[i].cpu().numpy(), de[tg], what="targets row %d" % i)
    # empty target list: nothing to write, no error
    empty = torch.empty(0, dtype=torch.float64, device=dev)
    bc.bc_dependencies(G, T(src, dev), bc.BC_OUT_TARGETS, empty,
                       targets=torch.empty(0, dtype=torch.int32, device=dev))
    with pytest.raises(bc.BcError) as e:
        bc.bc_dependencies(G, T(src, dev), bc.BC_OUT_TARGETS, torch.empty(k, dtype=torch.float64,
                                                                           device=dev),
                           targets=T(np.array([g.n], np.int32), dev))
    assert e.value.status == bc.BC_E_INVALID
    G.close()


def test_host_io_mode(dev):
    g = gg.config_graph("er2000")
    src = gg.philox_sources(4, 150, g.n)
    tg = gg.top_degree(g, 4)
    G = bc.Graph(g.row, g.col)
    say("host io: device reference")
    full_d, dist_d, sig_d = bc.dependencies(G, T(src, dev), bc.BC_OUT_FULL, dist=True, sigma=True)
    est_d = bc.adaptive_source(G, T(tg, dev), 3.0, 5, 2000)
    us = torch.empty(50, dtype=torch.int32, device=dev)
    vs = torch.empty(50, dtype=torch.int32, device=dev)
    bc.bc_draw_pairs(G, 2, 0, 50, us, vs)
    pd_d = bc.pair_dependencies(G, us, vs)
    ex_d = bc.exact(G)
    say("host io: host arrays")
    G.set_io(True)
    full = np.zeros(150 * g.n)
    dist = np.zeros(150 * g.n, np.int32)
    sm = np.zeros(150 * g.n)
    se = np.zeros(150 * g.n, np.int32)
    bc.bc_dependencies(G, src, bc.BC_OUT_FULL, full, dist, sm, se)
    assert np.array_equal(full, full_d.cpu().numpy().ravel())
    assert np.array_equal(dist, dist_d.cpu().numpy().ravel())
    assert np.array_equal(sm, sig_d[0].cpu().numpy().ravel())
    assert np.array_equal(se, sig_d[1].cpu().numpy().ravel())
    est, k, S, st = (np.zeros(4), np.zeros(4, np.int64), np.zeros(4), np.zeros(4, np.uint8))
    bc.bc_adaptive_source(G, tg, 3.0, 5, 2000, est, k, S, st)
    for a, b in zip((est, k, S, st), est_d):
        assert np.array_equal(a, b.cpu().numpy())
    hu = np.zeros(50, np.int32)
    hv = np.zeros(50, np.int32)
    bc.bc_draw_pairs(G, 2, 0, 50, hu, hv)
    assert np.array_equal(hu, us.cpu().numpy()) and np.array_equal(hv, vs.cpu().numpy())
    pd = np.zeros(50 * g.n)
    bc.bc_pair_dependencies(G, hu, hv, pd)
    assert np.array_equal(pd, pd_d.cpu().numpy().ravel())
    ex = np.zeros(g.n)
    bc.bc_exact(G, ex)
    assert np.array_equal(ex, ex_d.cpu().numpy())
    with pytest.raises(ValueError):
        bc.bc_exact(G, torch.empty(g.n, dtype=torch.float64, device=dev))
    G.close()


def test_int32_row_offsets_through_the_abi(dev):
    g = gg.rmat(12, 8, 0.57, 0.19, 0.19, seed=5)
    assert g.nnz < (1 << 31)
    lib = bc.load_library()
    row32 = np.ascontiguousarray(g.row, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    csr = bc._Csr(g.n, g.nnz, row32.ctypes.data, 0, col.ctypes.data)
    h = ctypes.c_void_p()
    say("int32 row offsets")
    assert lib.bc_graph_create(ctypes.byref(csr), None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                               ctypes.byref(h)) == bc.BC_OK
    src = gg.philox_sources(6, 200, g.n)
    s_t = T(src, dev)
    out32 = torch.empty(200 * g.n, dtype=torch.float64, device=dev)
    dist32 = torch.empty(200 * g.n, dtype=torch.int32, device=dev)
    rc = lib.bc_dependencies(h, ctypes.c_void_p(s_t.data_ptr()), 200, bc.BC_OUT_FULL,
                             ctypes.c_void_p(out32.data_ptr()), ctypes.c_void_p(dist32.data_ptr()),
                             None, None, None, 0)
    assert rc == bc.BC_OK, lib.bc_last_error()
    torch.cuda.synchronize()
    lib.bc_graph_destroy(h)
    G = bc.Graph(g.row, g.col)          # int64 offsets
    out64, dist64, _ = bc.dependencies(G, s_t, bc.BC_OUT_FULL, dist=True)
    G.close()
    assert torch.equal(out32.view(200, g.n), out64)
    assert torch.equal(dist32.view(200, g.n), dist64)
    for i in (0, 199):
        d, _, de = O.brandes(g, int(src[i]))
        assert np.array_equal(dist64[i].cpu().numpy(), d)
        assert_close(out64[i].cpu().numpy(), de, what="int32 rows %d" % i)
