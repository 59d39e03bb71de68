"""Whole small 2D Lawson solves in one workgroup (time loop on the device) against the
FP64 oracle and against the same solve launched kernel by kernel.

Bar: 1e-12 relative to the oracle (FP64, as every FP64 path); the two GPU paths sum the
mode products in different orders, so they agree to rounding, not bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import schemes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_15861_amd as m
    return m


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def run(mm, p, fused):
    ctx = mm.Context(0)
    ctx.set_small_fused(fused)
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    st = mm.mm_check(op)
    out = host(u)
    op.close()
    ctx.close()
    return st, out


@pytest.mark.parametrize("scheme", ["le", "l2b"])
@pytest.mark.parametrize("n", [(1, 1), (5, 7), (64, 64), (63, 63), (33, 64), (64, 17), (1, 64)])
def test_fused_matches_oracle_and_launched(mm, scheme, n):
    p = synth.smooth_problem(n, 41, tau=1e-3, steps=25, scheme=scheme, beta=(3.0, -2.0), beta_bar=(0.5, -0.25),
                             lam=0.9, r=(0.1, 0.7, -0.4, 0.2))
    st_f, u_f = run(mm, p, True)
    st_l, u_l = run(mm, p, False)
    assert st_f == mm.MM_OK and st_l == mm.MM_OK
    ref = S.solve(p)
    assert relerr(u_f, ref) <= 1e-12
    assert relerr(u_f, u_l) <= 1e-13


def test_fused_workload_c1(mm):
    p = synth.workload("2d_n63_le")
    st, u = run(mm, p, True)
    assert st == mm.MM_OK
    assert relerr(u, S.solve(p)) <= 1e-12


def test_fused_nonfinite_flag(mm):
    p = synth.smooth_problem((20, 18), 42, tau=1e-3, steps=3, scheme="l2b")
    p.u0 = p.u0.copy()
    p.u0[3, 4] = np.nan
    st, _ = run(mm, p, True)
    assert st == mm.MM_EUNSTABLE


def test_fused_in_graph_replay(mm):
    p = synth.smooth_problem((40, 36), 43, tau=1e-3, steps=9, scheme="le")
    outs = []
    for gs in (0, 4):
        ctx = mm.Context(0)
        ctx.set_graph_steps(gs)
        op = mm.setup_problem(ctx, p)
        u = dev(p.u0)
        mm.step(op, u, p.steps)
        outs.append(host(u))
        op.close()
        ctx.close()
    assert np.array_equal(outs[0], outs[1])
