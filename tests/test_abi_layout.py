"""The binding's ctypes structures against the C header (CPU only).

Every structure the library reads or writes through a caller's pointer
(tp_group, tp_plan_opts, tp_mesh, tp_solve_summary, tp_pcg_summary) must
have the same size and field offsets in include/tpfdm.h as in the binding:
a ctypes structure smaller than the C one lets tp_plan_opts_default (or a
summary write) run past the Python-owned memory and corrupt the host heap,
which surfaces as a segmentation fault far from its cause.  The header is
compiled with the host compiler and its sizeof/offsetof values compared.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2609_04534_amd import tpfdm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "tp_group": (tpfdm._Group, ["n", "layout_B", "nblocks", "h", "offset", "M", "P"]),
    "tp_plan_opts": (tpfdm._Opts, ["penalty_C", "persistent", "mapping", "blocks", "reserved"]),
    "tp_mesh": (tpfdm._Mesh, ["n", "layout_B", "cells", "basis", "h"]),
    "tp_solve_summary": (tpfdm._Summary, ["max_iters", "n_failed", "max_relres"]),
    "tp_pcg_summary": (tpfdm._PcgSummary, ["iterations", "converged", "relres"]),
}


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "tpfdm.h"', "int main(void) {"]
    for cname, (_, fields) in STRUCTS.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        name, key, val = line.split()
        layout[(name, key)] = int(val)
    return layout


def test_binding_structures_match_the_header(tmp_path):
    layout = _c_layout(tmp_path)
    for cname, (cls, fields) in STRUCTS.items():
        assert ctypes.sizeof(cls) == layout[(cname, "sizeof")], cname
        names = [f[0] for f in cls._fields_]
        assert names == fields, cname
        for f in fields:
            assert getattr(cls, f).offset == layout[(cname, f)], (cname, f)
