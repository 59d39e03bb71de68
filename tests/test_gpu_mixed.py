"""Mixed-precision contractions against the FP64 oracle.

Action bars (relative to max |oracle|, smooth data). A mode product of length K whose
operands are rounded to a t-bit significand (u_t = 2^-t) and summed in FP32 errs by
about (2 u_t + sqrt(K) u_24) |E||v| with random-walk accumulation; the heat-kernel
factors have row sums of |E| at most 1. Three passes per action give
    eps_action = 3 (2 u_t + sqrt(256) u_24):
    FP32   (t = 24): 3.2e-6        BF16x6 (t = 24): 3.2e-6
    BF16x3 (t = 16, hi + lo, lo*lo dropped ~ 2^-16): 9.4e-5

Solve bars. A whole solve carries one action error per step, and a stage that applies
g to an action's output without a following exponential (the last stage of Lawson2b)
multiplies the high-frequency part of that error by up to
    amp = 1 + 2 d tau (a_max - a_min) / h_min^2,
so eps_action * amp bounds the error; at 127^3 that is 158 times eps_action, and the
measured errors sit 14 to 100 times below it. The solve bars are therefore three times
the errors this build measures on MI355X (the kernels are deterministic), which fails
any several-fold loss of accuracy; the amplification bound is asserted as well. None
of these modes meets the stated targets of the 255^3 workload (1e-6 for FP32, 1e-9 for
the split modes) under Lawson2b: 24 or 16 significand bits times the amplification
(about 700 there) cannot. The exact-slice mode does (tests/test_gpu_full_size.py).
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo
from oracle import schemes as S

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24
EPS_ACTION = {"fp32": 3 * (2 * U24 + 16 * U24), "bf16x6": 3 * (2 * U24 + 16 * U24),
              "bf16x3": 3 * (2 * 2.0 ** -16 + 16 * U24)}


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
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("n", [(63, 63), (9, 13), (5, 6, 7), (130, 129, 127), (255, 255, 255)])
def test_mixed_exp_action(mm, ctx, prec, n):
    p = synth.smooth_problem(n, 3, tau=1e-3)
    op = mm.setup_problem(ctx, p, prec=prec)
    out = dev(np.zeros(p.shape))
    mm.mumode_expv(op, dev(p.u0), out)
    ref = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau).expv(1.0, p.u0)
    err = relerr(host(out), ref)
    op.close()
    print(f"{prec} {n} action err {err:.3e} (bar {EPS_ACTION[prec]:.1e})")
    assert err <= EPS_ACTION[prec]


# relative errors measured on MI355X (this build) for the cases of test_mixed_solve
MEASURED = {("fp32", "l2b", (48, 40, 36)): 1.33e-6, ("bf16x6", "l2b", (48, 40, 36)): 1.27e-6,
            ("bf16x3", "l2b", (48, 40, 36)): 4.73e-5, ("fp32", "le", (63, 63)): 6.50e-7,
            ("bf16x6", "le", (63, 63)): 3.76e-7, ("bf16x3", "le", (63, 63)): 2.81e-5,
            ("fp32", "etd2rk", (30, 28, 26)): 9.34e-7, ("bf16x6", "etd2rk", (30, 28, 26)): 8.99e-7,
            ("bf16x3", "etd2rk", (30, 28, 26)): 2.76e-5, ("fp32", "l2b", (127, 127, 127)): 2.78e-5,
            ("bf16x6", "l2b", (127, 127, 127)): 2.46e-5, ("bf16x3", "l2b", (127, 127, 127)): 1.07e-4}


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "bf16x3"])
@pytest.mark.parametrize("scheme,n,steps", [("l2b", (48, 40, 36), 20), ("le", (63, 63), 20),
                                            ("etd2rk", (30, 28, 26), 10), ("l2b", (127, 127, 127), 10)])
def test_mixed_solve(mm, ctx, prec, scheme, n, steps):
    p = synth.smooth_problem(n, 6, tau=1e-3, steps=steps, scheme=scheme, q=4)
    op = mm.setup_problem(ctx, p, prec=prec)
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    status = mm.mm_check(op)
    got = host(u)
    op.close()
    assert status == mm.MM_OK
    err = relerr(got, S.solve(p))
    bound = EPS_ACTION[prec] * amplification(p)
    bar = 3.0 * MEASURED[(prec, scheme, n)]
    print(f"{prec} {scheme} {n} x{steps} solve err {err:.3e} (bar {bar:.1e}, bound {bound:.1e})")
    assert err <= bound
    assert err <= bar
