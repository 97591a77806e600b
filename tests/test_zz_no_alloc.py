"""bc_dependencies_noalloc, the allocation-free call, against bc_dependencies.

Two calls in a row (the second with a smaller input) through the C ABI must
give bc_dependencies' results (1e-9 relative) and allocate nothing; path
counts beyond 2^1000 take the extended form inside the same array; oversized
graphs and host arrays are refused with BC_E_UNSUPPORTED.
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

O = oracle.load()
RTOL = 1e-9


def say(*a):
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def close(got, want, what):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    ok = np.abs(got - want) <= RTOL * np.abs(want)
    assert ok.all(), (what, int((~ok).sum()))


def noalloc(G, src, mode, out):
    """The entry point through the raw C ABI."""
    lib = bc.load_library()
    rc = lib.bc_dependencies_noalloc(G.handle, ctypes.c_void_p(src.data_ptr()), src.numel(),
                                     int(mode), ctypes.c_void_p(out.data_ptr()))
    if rc != bc.BC_OK:
        raise bc.BcError(rc, lib.bc_last_error().decode())


def test_two_calls_match_bc_dependencies(dev):
    g = gg.rmat(12, 16, 0.57, 0.19, 0.19, seed=9)
    G = bc.Graph(g.row, g.col)             # torch's allocator: its count must not move
    src1 = torch.from_numpy(gg.philox_sources(21, 300, g.n)).to(dev)
    src2 = torch.from_numpy(gg.philox_sources(22, 70, g.n)).to(dev)
    out1 = torch.empty(300 * g.n, dtype=torch.float64, device=dev)
    out2 = torch.empty(g.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    say("noalloc call 1: FULL, 300 sources")
    noalloc(G, src1, bc.BC_OUT_FULL, out1)
    say("noalloc call 2: SUM, 70 sources")
    noalloc(G, src2, bc.BC_OUT_SUM, out2)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    say("reference calls")
    ref1, _, _ = bc.dependencies(G, src1, bc.BC_OUT_FULL)
    ref2, _, _ = bc.dependencies(G, src2, bc.BC_OUT_SUM)
    close(out1.view(300, g.n).cpu().numpy(), ref1.cpu().numpy(), "call 1 vs bc_dependencies")
    close(out2.cpu().numpy(), ref2.cpu().numpy(), "call 2 vs bc_dependencies")
    s1 = src1.cpu().numpy()
    for i in (0, 151, 299):
        close(out1.view(300, g.n)[i].cpu().numpy(), O.brandes(g, int(s1[i]))[2],
              "call 1 row %d vs oracle" % i)
    _, want2 = O.dependencies(g, src2.cpu().numpy(), full=False, total=True)
    close(out2.cpu().numpy(), want2, "call 2 vs oracle")
    # the same calls again, now after the allocating call ran on this graph
    say("noalloc again, after bc_dependencies")
    out3 = torch.empty(70 * g.n, dtype=torch.float64, device=dev)
    noalloc(G, src2, bc.BC_OUT_FULL, out3)
    ref3, _, _ = bc.dependencies(G, src2, bc.BC_OUT_FULL)
    close(out3.view(70, g.n).cpu().numpy(), ref3.cpu().numpy(), "call 3 vs bc_dependencies")
    G.close()


def test_extended_counts_in_the_scratch(dev):
    # 260 layers of 16 vertices, consecutive layers completely joined: from
    # layer 0, path counts grow 16-fold per layer, past 2^1000 at the end
    layers, width = 260, 16
    a, b = [], []
    for L in range(layers - 1):
        for i in range(width):
            for j in range(width):
                a.append(L * width + i)
                b.append((L + 1) * width + j)
    g = gg.from_edges(layers * width, a, b, "layers")
    G = bc.Graph(g.row, g.col)
    src = torch.tensor([0, 5, 2100, 4159, 3], dtype=torch.int32, device=dev)
    out = torch.empty(5 * g.n, dtype=torch.float64, device=dev)
    say("noalloc extended counts")
    noalloc(G, src, bc.BC_OUT_FULL, out)
    assert G.stats()["extended"] == 1
    out2 = torch.empty(g.n, dtype=torch.float64, device=dev)
    noalloc(G, src[:2].contiguous(), bc.BC_OUT_SUM, out2)
    ref, _, _ = bc.dependencies(G, src, bc.BC_OUT_FULL)
    close(out.view(5, g.n).cpu().numpy(), ref.cpu().numpy(), "extended vs bc_dependencies")
    for i, s in enumerate(src.cpu().numpy()):
        close(out.view(5, g.n)[i].cpu().numpy(), O.brandes(g, int(s))[2], "extended row %d" % i)
    close(out2.cpu().numpy(), ref[:2].sum(0).cpu().numpy(), "extended sum")
    G.close()


def test_refusals(dev):
    g = gg.path(500000)
    G = bc.Graph(g.row, g.col)
    src = torch.zeros(4, dtype=torch.int32, device=dev)
    say("noalloc oversized")
    for mode, size in ((bc.BC_OUT_FULL, 4 * g.n), (bc.BC_OUT_SUM, g.n)):
        with pytest.raises(bc.BcError) as e:
            noalloc(G, src, mode, torch.empty(size, dtype=torch.float64, device=dev))
        assert e.value.status == bc.BC_E_UNSUPPORTED and "too large" in str(e.value)
    G.close()
    g = gg.er(300, 0.02, seed=5)
    G = bc.Graph(g.row, g.col)
    lib = bc.load_library()
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    with pytest.raises(bc.BcError) as e:
        noalloc(G, torch.tensor([0, 300], dtype=torch.int32, device=dev), bc.BC_OUT_SUM, out)
    assert e.value.status == bc.BC_E_INVALID
    assert lib.bc_dependencies_noalloc(G.handle, None, 1, bc.BC_OUT_SUM, None) == bc.BC_E_INVALID
    assert lib.bc_dependencies_noalloc(G.handle, ctypes.c_void_p(src.data_ptr()), 1,
                                       bc.BC_OUT_TARGETS,
                                       ctypes.c_void_p(out.data_ptr())) == bc.BC_E_INVALID
    G.set_io(True)
    with pytest.raises(bc.BcError) as e:
        noalloc(G, src, bc.BC_OUT_SUM, out)
    assert e.value.status == bc.BC_E_UNSUPPORTED
    G.close()
