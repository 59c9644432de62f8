"""The binding's structures and flags match the C headers.

A small C program built with the host compiler from include/ipi.h and
include/ipi_server.h prints every field offset and the size of each struct
the binding mirrors, and the create flags; the ctypes definitions in
paper_2507_22538_amd/ipi.py must agree field for field (a field added to a
header and not to the binding, or the reverse, fails here).
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2507_22538_amd import ipi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [ipi.ipi_mdp_desc, ipi.ipi_solve_opts, ipi.ipi_solve_info, ipi.ipi_tuning, ipi.ipi_server_opts,
           ipi.ipi_latency]
FLAGS = ["IPI_DEVICE_PTRS", "IPI_VAL_FP32", "IPI_FP32_ORIGIN", "IPI_BORROW", "IPI_NO_VALIDATE",
         "IPI_VAL_FP32_ONLY", "IPI_VAL_SPLIT"]


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ipi.h"', '#include "ipi_server.h"',
             "int main(void) {"]
    for st in STRUCTS:
        n = st.__name__
        lines.append(f'  printf("{n} sizeof %zu\\n", sizeof({n}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{n} {f} %zu %zu\\n", offsetof({n}, {f}), sizeof((({n}*)0)->{f}));')
    for fl in FLAGS:
        lines.append(f'  printf("flag {fl} %u\\n", (unsigned){fl});')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return [ln.split() for ln in out.splitlines()]


def test_structs_and_flags_match_headers(tmp_path):
    rows = _c_layout(tmp_path)
    seen = 0
    for r in rows:
        if r[0] == "flag":
            assert getattr(ipi, r[1]) == int(r[2]), r
            seen += 1
            continue
        st = getattr(ipi, r[0])
        if r[1] == "sizeof":
            assert ctypes.sizeof(st) == int(r[2]), r
        else:
            fld = getattr(st, r[1])
            assert (fld.offset, fld.size) == (int(r[2]), int(r[3])), r
        seen += 1
    assert seen == len(FLAGS) + sum(1 + len(st._fields_) for st in STRUCTS)
