"""Host-side checks of the Python binding (no GPU needed): the library shares torch's HIP
runtime whatever the import order, and every call refuses buffers whose size does not
match the problem before anything reaches the kernels."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import paper_2303_15861_amd as mm
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_shares_torchs_hip_runtime():
    # a fresh process that asks for the library before it has imported torch itself
    code = ("import paper_2303_15861_amd as mm; mm.lib(); "
            "print(len(mm._hip_runtimes()), sorted(mm._hip_runtimes()))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    count, files = out.stdout.split(" ", 1)
    assert count == "1", files
    assert "torch" in files, files


def test_coefficient_size():
    assert mm.coefficient_size(3, (4, 5, 6), False) == 6 * 7 * 8
    assert mm.coefficient_size(2, (4, 5, 1), False) == 6 * 7
    assert mm.coefficient_size(2, (4, 5, 1), True) == 2 * 20


def fake_operator(n):
    """An Operator object with a problem size but no library handle behind it."""
    ctx = object.__new__(mm.Context)
    ctx._h, ctx.device = None, 0
    op = object.__new__(mm.Operator)
    op.ctx, op._h, op.d, op.n = ctx, 1, len(n), tuple(n)
    op.dof = int(np.prod(n))
    return op


@pytest.mark.parametrize("n", [(7, 6, 5), (9, 4)])
def test_grid_buffers_of_the_wrong_size_are_refused(n):
    op = fake_operator(n)
    dof = int(np.prod(n))
    for bad in (dof - 1, dof + 1, 1):
        with pytest.raises(ValueError, match="needs"):
            op.grid(torch.zeros(bad, dtype=torch.float64), "u")
    # the right size passes the size check and then needs a GPU tensor
    with pytest.raises(TypeError):
        op.grid(torch.zeros(dof, dtype=torch.float64), "u")
    with pytest.raises(ValueError, match="closed"):
        op._h = None
        op.grid(torch.zeros(dof, dtype=torch.float64), "u")


def test_setup_refuses_a_short_coefficient():
    ctx = object.__new__(mm.Context)
    ctx._h, ctx.device = None, 0
    a = torch.zeros(6 * 7 * 8 - 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="diffusion coefficient"):
        mm.mumode_setup(ctx, 3, (4, 5, 6), a, (0, 0, 0), (0, 0, 0, 0), 1e-3)


class _NoServer:
    """Stands in for a server: submit must fail before any library call."""
    _h = None
    _shapes = {}


def test_submit_refuses_wrong_sizes():
    p = synth.smooth_problem((6, 5, 4), 0, tau=1e-3, steps=2)
    short_u = synth.smooth_problem((6, 5, 4), 0, tau=1e-3, steps=2)
    short_u.u0 = short_u.u0.reshape(-1)[:-1]
    with pytest.raises(ValueError, match="u0"):
        mm.solve_submit(_NoServer(), short_u)
    short_a = synth.smooth_problem((6, 5, 4), 0, tau=1e-3, steps=2)
    short_a.a = short_a.a.reshape(-1)[:-3]
    with pytest.raises(ValueError, match="a has"):
        mm.solve_submit(_NoServer(), short_a)
    assert p.a.size == mm.coefficient_size(3, p.n, False)
