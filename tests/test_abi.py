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


def _c_layout(struct, fields):
    """sizeof and field offsets of a header struct, from a C program built with gcc."""
    import subprocess
    import tempfile
    body = "\n".join(f'  printf("%s %zu\\n", "{f}", offsetof({struct}, {f}));' for f in fields)
    src = f"""#include <stddef.h>
#include <stdio.h>
#include "mumode.h"
int main(void) {{
  printf("sizeof %zu\\n", sizeof({struct}));
{body}
  return 0;
}}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


@pytest.mark.parametrize("cls,struct", [("MMProblem", "mm_problem"), ("MMRequest", "mm_request"),
                                        ("MMStats", "mm_stats")])
def test_binding_structs_match_the_header(cls, struct):
    """The ctypes mirrors of the ABI structs have the header's size and field offsets (the
    binding's field names map to the header's: lam -> lambda)."""
    import shutil
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    import paper_2303_15861_amd as mm
    S = getattr(mm, cls)
    cnames = {"lam": "lambda"}
    fields = [f for f, _ in S._fields_]
    lay = _c_layout(struct, [cnames.get(f, f) for f in fields])
    assert lay["sizeof"] == ctypes.sizeof(S)
    for f in fields:
        assert lay[cnames.get(f, f)] == getattr(S, f).offset, f
