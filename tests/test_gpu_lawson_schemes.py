"""The paper's other Lawson schemes on the GPU (Sec. 2: stabilized Lawson-Euler,
Lawson2a, stabilized Lawson2 with alpha = 0.327) against the FP64 oracle, which the CPU
tests pin to the stability functions of Sec. 2 and to the printed errors of Figure
fig:ad1dex0_diffdeltaa. These schemes are meant for lambda < 1 extraction, so the cases
use lambda in (0.3, 1) and a nonzero extracted velocity.

Bars: FP64 1e-12 relative; the sliced precision against the sliced oracle with the
last-digit-flip bar of the sliced tests times the stiffness amplification.
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo, sliced
from oracle import schemes as S

pytestmark = pytest.mark.gpu


def amplification(p):
    h = 1.0 / (max(p.n) + 1)
    return 1.0 + 2 * p.d * p.tau * (float(p.a.max()) - float(p.a.min())) / h ** 2


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_15861_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mm):
    c = mm.Context(0)
    yield c
    c.close()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def problem(scheme, n, steps, lam, seed):
    d = len(n)
    return synth.smooth_problem(n, seed, tau=1e-3, steps=steps, scheme=scheme, lam=lam,
                                beta=(3.0, -2.0, 1.5)[:d], beta_bar=(1.0, -0.5, 0.5)[:d])


@pytest.mark.parametrize("scheme", ["sle", "l2a", "sl2"])
@pytest.mark.parametrize("n,lam", [((63, 63), 0.5), ((41, 37), 0.35), ((24, 20, 18), 0.5), ((17, 19, 21), 0.8)])
def test_fp64_solve(mm, ctx, scheme, n, lam):
    p = problem(scheme, n, 12, lam, 31)
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    assert mm.mm_check(op) == mm.MM_OK
    got = host(u)
    op.close()
    assert relerr(got, S.solve(p)) <= 1e-12


@pytest.mark.parametrize("scheme", ["sle", "l2a", "sl2"])
def test_sliced_solve(mm, ctx, scheme):
    S_ = 6
    p = problem(scheme, (22, 19, 17), 6, 0.5, 32)
    op = mm.setup_problem(ctx, p, prec=f"sliced{S_}")
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    got = host(u)
    op.close()
    ref = sliced.solve(p, S_)
    oop = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau)
    emax = max(float(np.max(np.abs(M))) for c in (1.0, 0.5, S.ALPHA_SL2) for M in oop.factors(c))
    bar = (1e-12 + 128 * 2.0 ** (-8 * S_) * emax) * amplification(p)
    assert np.max(np.abs(got - ref)) <= bar * float(np.max(np.abs(ref)))


def test_extra_factors(mm, ctx):
    """Lawson2a stores exp(tau A / 2), stabilized Lawson2 also exp(alpha tau A)."""
    p = problem("sl2", (15, 13, 11), 1, 0.5, 33)
    op = mm.setup_problem(ctx, p)
    oop = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau)
    for j, c in ((0, 1.0), (1, 0.5), (2, S.ALPHA_SL2)):
        for mu in range(3):
            E = op.factor(mu, j)
            R = oop.factors(c)[mu]
            assert np.max(np.abs(E - R)) <= 1e-12 * np.max(np.abs(R)), (j, mu)
    op.close()
