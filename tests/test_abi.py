"""The C-ABI library loads on a machine without a GPU and exports every
function include/nhp.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nhp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_declares_the_pipeline():
    names = declared_functions()
    for n in ("plan_create", "render_cspace", "sweep_n_turns", "extract_path", "plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2306_01301_amd import planner

    if not os.path.exists(planner.LIB_PATH):
        pytest.fail("libnhp.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(planner.LIB_PATH)
    for n in declared_functions():
        assert hasattr(L, n), n
        assert n in planner.SIGNATURES, n


def test_workspace_bytes_and_param_checks_need_no_gpu():
    from paper_2306_01301_amd import planner

    p = planner.make_params(512, 512, 12.0, [1024] * 6)
    nb = planner.workspace_bytes(p)
    nr = 512 ** 3
    assert 5 * nr <= nb < 5 * nr + 8 * 2 ** 20
    bad = planner.make_params(500, 512, 12.0, [1024] * 6)  # not a multiple of 8
    assert planner.workspace_bytes(bad) == 0
    assert b"multiple of 8" in planner.lib().plan_last_error()
    bad = planner.make_params(64, 64, -1.0, [1024] * 6)
    assert planner.workspace_bytes(bad) == 0


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of nhp_params / nhp_step have the C compiler's layout."""
    import subprocess

    from paper_2306_01301_amd import planner

    fields = {"nhp_params": [f[0] for f in planner.NhpParams._fields_],
              "nhp_step": [f[0] for f in planner.NhpStep._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nhp.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append('printf("%%zu\\n", sizeof(%s));' % st)
        for f in fs:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (st, f))
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for cls in (planner.NhpParams, planner.NhpStep):
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f[0]).offset for f in cls._fields_]
    assert got == want
