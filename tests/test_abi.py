"""CPU checks of the C ABI library: it loads and exports every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2303_15861_amd", "libmumode.so")
HEADER = os.path.join(ROOT, "include", "mumode.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mumode_setup", "lawson_step", "erk_step", "remainder_eval", "solve_submit",
                     "solve_poll", "mumode_expv", "mumode_phi1v"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_declares_every_export():
    import paper_2303_15861_amd as mm
    assert sorted(mm.EXPORTS) == declared_functions()
    lib = mm.load_library()
    assert lib.mm_version().decode().startswith("mumode")


def test_binding_fails_loudly_without_library(tmp_path):
    import paper_2303_15861_amd as mm
    with pytest.raises(ImportError):
        mm.load_library(str(tmp_path / "libmumode.so"))
