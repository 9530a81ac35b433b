"""The ctypes mirrors of the C ABI's structs (paper_2111_10743_amd.lb) have
the sizes and field offsets that a C compiler gives the declarations in
include/lb.h (compiled here with gcc; no GPU needed)."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "lb_opts": "Opts",
    "lb_solve_info": "SolveInfo",
    "lb_sizes": "Sizes",
    "lb_tree_info": "TreeInfo",
    "lb_tune_info": "TuneInfo",
}


def test_struct_layouts_match_header():
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_2111_10743_amd import lb
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lb.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(lb, pyname)
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "abi.c")
        exe = os.path.join(d, "abi")
        with open(src, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    c = {}
    for line in out.splitlines():
        sname, key, val = line.split()
        c[(sname, key)] = int(val)
    for cname, pyname in STRUCTS.items():
        cls = getattr(lb, pyname)
        assert ctypes.sizeof(cls) == c[(cname, "sizeof")], cname
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == c[(cname, fname)], (cname, fname)
