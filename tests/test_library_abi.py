"""CPU-side checks of the C-ABI library: it loads and exports every symbol that
include/imsmg.h and include/imsmg_gen.h declare (no GPU compute is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_10977_amd", "lib")


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(imsmg_\w+)\s*\(", txt))
    return sorted(names)


@pytest.mark.parametrize("header,so", [("imsmg.h", "libimsmg.so"), ("imsmg_gen.h", "libimsmg_gen.so")])
def test_library_exports_declared_symbols(header, so):
    path = os.path.join(LIB, so)
    if not os.path.exists(path):
        pytest.skip(f"{so} not built")
    lib = ctypes.CDLL(path)
    names = _declared(header)
    assert len(names) >= 8
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_solver_symbol():
    from paper_1903_10977_amd import solver
    assert sorted(solver.SYMBOLS) == _declared("imsmg.h")


def test_product_path_has_no_oracle_import():
    """The product package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_1903_10977_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
