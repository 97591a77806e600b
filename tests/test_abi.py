"""The C-ABI library loads on the CPU host and exports every declared symbol.

No compute calls here (no GPU); argument checks that fail before any device
work are exercised where they need no device.
"""
import ctypes
import os
import re

import pytest

import paper_1608_04472_amd as bc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bcmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bc_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_calls():
    names = declared_functions()
    for want in ("bc_exact", "bc_dependencies", "bc_adaptive_source", "bc_adaptive_pair",
                 "bc_graph_create", "bc_graph_destroy", "bc_last_error"):
        assert want in names
    assert sorted(bc.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_loads():
    lib = bc.load_library()
    assert lib.bc_last_error() in (b"",)


def test_invalid_csr_rejected_before_device_work():
    import numpy as np
    lib = bc.load_library()
    # asymmetric: edge 0->1 without 1->0
    row = np.array([0, 1, 1], dtype=np.int64)
    col = np.array([1], dtype=np.int32)
    csr = bc._Csr(2, 1, row.ctypes.data, 1, col.ctypes.data)
    h = ctypes.c_void_p()
    rc = lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h))
    assert rc == bc.BC_E_INVALID
    assert b"symmetric" in lib.bc_last_error()
    # self-loop
    row = np.array([0, 1], dtype=np.int64)
    col = np.array([0], dtype=np.int32)
    csr = bc._Csr(1, 1, row.ctypes.data, 1, col.ctypes.data)
    assert lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h)) == bc.BC_E_INVALID
    # unsorted row
    row = np.array([0, 2, 3, 4], dtype=np.int64)
    col = np.array([2, 1, 0, 0], dtype=np.int32)
    csr = bc._Csr(3, 4, row.ctypes.data, 1, col.ctypes.data)
    assert lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h)) == bc.BC_E_INVALID
    # n = 0
    csr = bc._Csr(0, 0, row.ctypes.data, 1, None)
    assert lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h)) == bc.BC_E_INVALID


def test_null_arguments_rejected():
    lib = bc.load_library()
    assert lib.bc_exact(None, None) == bc.BC_E_INVALID
    assert lib.bc_dependencies(None, None, 0, 0, None, None, None, None, None, 0) == bc.BC_E_INVALID
    assert lib.bc_adaptive_source(None, None, 0, 2.0, 1, 1, None, None, None, None) \
        == bc.BC_E_INVALID
    assert lib.bc_graph_configure(None, None) == bc.BC_E_INVALID


def test_int32_row_offsets_validated_on_the_host():
    import numpy as np
    lib = bc.load_library()
    h = ctypes.c_void_p()
    # asymmetric with int32 offsets
    row = np.array([0, 1, 1], dtype=np.int32)
    col = np.array([1], dtype=np.int32)
    csr = bc._Csr(2, 1, row.ctypes.data, 0, col.ctypes.data)
    assert lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h)) == bc.BC_E_INVALID
    assert b"symmetric" in lib.bc_last_error()
    # row[n] != nnz
    row = np.array([0, 1, 3], dtype=np.int32)
    col = np.array([1, 0], dtype=np.int32)
    csr = bc._Csr(2, 2, row.ctypes.data, 0, col.ctypes.data)
    assert lib.bc_graph_create(ctypes.byref(csr), None, None, ctypes.byref(h)) == bc.BC_E_INVALID
    # the binding keeps int32 offsets as int32
    csr, keep = bc._csr_arrays(np.array([0, 1, 2], dtype=np.int32), np.array([1, 0]))
    assert csr.row_is_i64 == 0 and keep[0].dtype == np.int32
    csr, keep = bc._csr_arrays(np.array([0, 1, 2]), np.array([1, 0]))
    assert csr.row_is_i64 == 1


def test_allocator_needs_both_functions():
    import numpy as np
    lib = bc.load_library()
    row = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    csr = bc._Csr(2, 2, row.ctypes.data, 1, col.ctypes.data)
    half = bc._Allocator(bc._ALLOC_FN(lambda size, ctx: None), bc._FREE_FN(), None)
    h = ctypes.c_void_p()
    assert lib.bc_graph_create(ctypes.byref(csr), ctypes.byref(half), None,
                               ctypes.byref(h)) == bc.BC_E_INVALID
    assert b"allocator" in lib.bc_last_error()
    s = ctypes.c_void_p()
    assert lib.bc_server_create(1 << 30, 64, ctypes.byref(half), None,
                                ctypes.byref(s)) == bc.BC_E_INVALID


def test_server_arguments_checked_before_device_work():
    lib = bc.load_library()
    s = ctypes.c_void_p()
    assert lib.bc_server_create(1 << 30, 96, None, None, ctypes.byref(s)) == bc.BC_E_INVALID
    assert lib.bc_server_create(0, 64, None, None, ctypes.byref(s)) == bc.BC_E_INVALID
    assert lib.bc_server_graph_width(None, 0, None, None) == bc.BC_E_INVALID
    assert lib.bc_graph_set_io(None, 1) == bc.BC_E_INVALID


def test_weights_validated_on_the_host():
    import numpy as np
    import graphgen as gg
    lib = bc.load_library()
    g = gg.with_weights(gg.path(5), 3, seed=1)
    csr, keep = bc._csr_arrays(g.row, g.col)
    h = ctypes.c_void_p()

    def create(w, directed=0):
        w = np.ascontiguousarray(w, dtype=np.int32)
        return lib.bc_graph_create_weighted(ctypes.byref(csr), w.ctypes.data, directed, None,
                                            None, ctypes.byref(h))

    zero = g.w.copy()
    zero[3] = 0
    assert create(zero) == bc.BC_E_INVALID
    assert b"positive" in lib.bc_last_error()
    asym = g.w.copy()
    asym[0] += 1
    assert create(asym) == bc.BC_E_INVALID
    assert b"different weights" in lib.bc_last_error()
    assert create(np.full(g.nnz, 1 << 28)) == bc.BC_E_INVALID
    assert lib.bc_graph_create_weighted(ctypes.byref(csr), None, 0, None, None,
                                        ctypes.byref(h)) == bc.BC_E_INVALID
