"""CPU checks of the C ABI library: it loads and exports every declared entry point."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (the HIP runtime the library shares, mapped before it is loaded)

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
                                        ("MMStats", "mm_stats"),
                                        ("MMServerCounters", "mm_server_counters")])
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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_entry_points_reject_null_handles_before_any_device_call():
    """Every entry point checks its handles and pointers first and returns MM_EINVAL (or
    the documented neutral value) without touching the device, so these calls are safe on
    a machine with no GPU."""
    import paper_2303_15861_amd as mm
    lib = mm.load_library()
    EINVAL = mm.MM_EINVAL
    out = ctypes.c_void_p(123)
    assert lib.mm_ctx_create(0, None) == EINVAL
    assert lib.mm_last_error(None).decode() == "null context"
    prob = mm.MMProblem()
    assert lib.mumode_setup(None, ctypes.byref(prob), 0.1, 0, 0, 0, 0, 0, ctypes.byref(out)) == EINVAL
    assert lib.mumode_info(None, None, None) == EINVAL
    assert lib.mumode_get_factor(None, 0, 0, None) == EINVAL
    assert lib.remainder_eval(None, None, None, None, None, None) == EINVAL
    assert lib.mumode_expv(None, None, 0, None, None, None) == EINVAL
    assert lib.mumode_phi1v(None, None, None, None, None) == EINVAL
    assert lib.lawson_step(None, None, None, 1, None) == EINVAL
    assert lib.erk_step(None, None, None, 1, None) == EINVAL
    assert lib.mm_check(None, None, None) == EINVAL
    assert lib.mm_synchronize(None) == EINVAL
    assert lib.mm_timing_enable(None, 1) == EINVAL
    assert lib.mm_set_gemm_tile(None, 64) == EINVAL
    assert lib.mm_set_graph_steps(None, 1) == EINVAL
    assert lib.mm_set_small_fused(None, 1) == EINVAL
    assert lib.mm_set_sliced_chain(None, 1) == EINVAL
    assert lib.mm_set_fold(None, 1) == EINVAL
    assert lib.mm_timing_read(None, 0, None, None, None) == EINVAL
    lib.mumode_destroy(None)
    srv = ctypes.c_void_p(123)
    assert lib.mm_server_create(0, 0, 0, ctypes.byref(srv)) == EINVAL   # max_active < 1
    assert srv.value is None                                             # cleared on failure
    assert lib.mm_server_create(0, 4, 0, None) == EINVAL
    rid = ctypes.c_uint64(0)
    req = mm.MMRequest()
    assert lib.solve_submit(None, ctypes.byref(req), ctypes.byref(rid)) == EINVAL
    assert lib.solve_poll(None, 1, None, None) == EINVAL
    assert lib.mm_server_clock(None) == 0.0
    assert lib.mm_server_read_counters(None, None) == EINVAL
    assert lib.lawson_step_batch(None, None, None, 1, 1, None) == EINVAL
    lib.mm_server_destroy(None)
