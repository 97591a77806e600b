"""The binding's ctypes structures against the C header: every structure the
binding passes through the ABI has the same size, and every field the same
offset, as a C compiler lays them out from include/bcmi.h (gcc, host ABI)."""
import ctypes
import os
import subprocess

import pytest

import paper_1608_04472_amd as bc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("_Csr", "bc_csr"), ("_Config", "bc_config"), ("_Stats", "bc_stats"),
         ("_KProf", "bc_kernel_profile"), ("_Query", "bc_query"), ("_Result", "bc_result"),
         ("_ServerStats", "bc_server_stats"), ("_Allocator", "bc_allocator")]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bcmi.h"', "int main(void) {"]
    for py, c in PAIRS:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (c, c))
        for f, _ in getattr(bc, py)._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (c, f, c, f))
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        struct, field, value = line.split()
        out[(struct, field)] = int(value)
    return out


@pytest.mark.parametrize("py,c", PAIRS, ids=[p[1] for p in PAIRS])
def test_structure_matches_the_header(c_layout, py, c):
    cls = getattr(bc, py)
    assert ctypes.sizeof(cls) == c_layout[(c, "size")], (c, ctypes.sizeof(cls))
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[(c, f)], (c, f)
