"""The ctypes mirrors of the C ABI structs match include/imsmg.h.

A small C program compiled with the host compiler prints sizeof and the
offset of every field that the Python binding declares; a field missing from
the header fails the compile, a moved or resized one fails the comparison.
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "imsmg_csr": "Csr",
    "imsmg_patches": "Patches",
    "imsmg_elements": "Elements",
    "imsmg_lattice": "Lattice",
    "imsmg_options": "Options",
    "imsmg_info": "Info",
    "imsmg_level_stats": "LevelStats",
}


def test_ctypes_structs_match_the_header(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_1903_10977_amd import solver as S
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "imsmg.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        py = getattr(S, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, pyname in STRUCTS.items():
        py = getattr(S, pyname)
        assert C.sizeof(py) == got[(cname, "size")], cname
        for f in py._fields_:
            assert getattr(py, f[0]).offset == got[(cname, f[0])], (cname, f[0])
