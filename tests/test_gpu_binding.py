"""Binding life cycle on the GPU, each case in a fresh process: a context made before
any torch GPU call leaves torch's device usable (one shared HIP runtime), and objects
left open at interpreter exit (an operator, a server, device tensors) are released by
the binding's exit handler without an abort."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run(code):
    print(f"[subprocess] {code[:80]}...", flush=True)
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=240)
    print(out.stdout[-2000:], out.stderr[-2000:], flush=True)
    return out


def test_context_before_torch_gpu_use():
    code = """
import paper_2303_15861_amd as mm
ctx = mm.Context(0)                # the first GPU call of the process
import torch
assert torch.cuda.is_available()
x = torch.ones(1000, dtype=torch.float64, device="cuda")
assert float(x.sum()) == 1000.0
ctx.close()
print("ok")
"""
    out = run(code)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok")


def test_open_objects_at_exit():
    code = """
import torch, numpy as np
import paper_2303_15861_amd as mm, synth
p = synth.smooth_problem((20, 18, 16), 3, tau=1e-3, steps=3)
ctx = mm.Context(0)
op = mm.setup_problem(ctx, p)
u = torch.from_numpy(p.u0.copy()).to("cuda")
mm.lawson_step(op, u, 3)                        # work still queued at exit
srv = mm.Server(0, max_active=2)
st, rid = mm.solve_submit(srv, p)               # a request still running at exit
keep = [op, u, srv, ctx]
cycle = [keep]
cycle.append(cycle)                              # held by a reference cycle as well
print("leaving", st)
"""
    out = run(code)
    assert out.returncode == 0, out.stderr
    assert "leaving 0" in out.stdout
