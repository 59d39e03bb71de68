"""Exact-slice contractions (precision "slicedS") on the GPU against the sliced oracle.

Both sides evaluate the same definition (digits of each factor row and grid fiber,
exact integer level sums, FP64 combination), but each with its own FP64 factors
(device Pade vs the sine-transform closed form) and its own stencil rounding, so a
value that lies within ~1e-16 of a digit boundary can round to neighbouring last
digits on the two sides. Each such flip moves a value by one unit of its last digit,
2^(e+2-8S) <= 8 * 2^(-8S) times its row or fiber maximum; the bar allows sixteen of
them on top of FP64 rounding:
    action:  |gpu - oracle| <= (1e-12 + 128 * 2^(-8S) * max|E|) * max|V|.
A whole Lawson2b solve multiplies such differences by at most the stiffness
amplification of its last stage (see the mixed-precision tests). Against the exact
(unsliced) oracle the bar is the error bound of the definition,
    3 * 2^(-8S) * 16 S * K * max|E| * max|V| per action.
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo, sliced
from oracle import schemes as Sch

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


def oracle_op(p):
    return expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau)


# (300, 270) and (20, 9, 290): contractions longer than 256 (the grid split's looped row
# path and its two-pass column path)
CASES = [((9, 13), 3), ((9, 13), 7), ((200, 130), 5), ((300, 270), 6), ((1, 1, 1), 4), ((5, 6, 7), 6),
         ((70, 65, 66), 3), ((70, 65, 66), 4), ((70, 65, 66), 5), ((70, 65, 66), 6), ((70, 65, 66), 7),
         ((130, 129, 127), 6), ((20, 9, 290), 7)]


def flip_bar(S, emax):
    return 1e-12 + 128 * 2.0 ** (-8 * S) * emax


@pytest.mark.parametrize("n,S", CASES)
def test_action_matches_sliced_oracle(mm, ctx, n, S):
    p = synth.smooth_problem(n, 11, tau=1e-3, beta_bar=(1.0, -0.5, 0.25)[: len(n)])
    V = np.random.default_rng(12).standard_normal(p.shape)
    op = mm.setup_problem(ctx, p, prec=f"sliced{S}")
    out = dev(np.zeros(p.shape))
    mm.mumode_expv(op, dev(V), out)
    got = host(out)
    op.close()
    oop = oracle_op(p)
    mats = oop.factors(1.0)
    emax = max(float(np.max(np.abs(M))) for M in mats)
    vmax = float(np.max(np.abs(V)))
    ref_sliced = sliced.tucker(V, mats, S)
    assert np.max(np.abs(got - ref_sliced)) <= flip_bar(S, emax) * vmax
    ref = oop.expv(1.0, V)
    K = max(p.n)
    assert np.max(np.abs(got - ref)) <= 3 * 2.0 ** (-8 * S) * 16 * S * K * emax * vmax + 1e-13 * vmax


@pytest.mark.parametrize("scheme,n,steps,S", [("le", (63, 63), 100, 6), ("l2b", (24, 20, 18), 20, 4),
                                              ("l2b", (24, 20, 18), 20, 7), ("l2b", (31, 29, 30), 10, 6)])
def test_lawson_solve_matches_sliced_oracle(mm, ctx, scheme, n, steps, S):
    p = synth.smooth_problem(n, 13, tau=1e-3, steps=steps, scheme=scheme, beta=(4.0, -3.0, 2.0)[: len(n)])
    op = mm.setup_problem(ctx, p, prec=f"sliced{S}")
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    assert mm.mm_check(op) == mm.MM_OK
    got = host(u)
    op.close()
    ref = sliced.solve(p, S)
    emax = max(float(np.max(np.abs(M))) for M in oracle_op(p).factors(1.0))
    scale = float(np.max(np.abs(ref)))
    assert np.max(np.abs(got - ref)) <= flip_bar(S, emax) * amplification(p) * scale


# (22, 19, 70): the stacked last mode contracts (q + 1) 70 = 350 > 256 values per fiber
@pytest.mark.parametrize("scheme,n", [("etd2rk", (22, 19, 17)), ("erk2p1f", (22, 19, 17)), ("etd2rk", (22, 19, 70))])
def test_erk_solve_within_slicing_bound(mm, ctx, scheme, n):
    S = 6
    p = synth.smooth_problem(n, 14, tau=1e-3, steps=8, scheme=scheme, beta=(2.0, 1.0, -1.0))
    op = mm.setup_problem(ctx, p, prec=f"sliced{S}")
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    got = host(u)
    op.close()
    ref = Sch.solve(p)
    K = (p.q + 1) * max(p.n)
    eps = 3 * 2.0 ** (-8 * S) * 16 * S * K
    assert np.max(np.abs(got - ref)) <= (eps * amplification(p) + 1e-12) * float(np.max(np.abs(ref)))


def test_digit_count_validated(mm, ctx):
    from ctypes import byref, c_void_p
    p = synth.smooth_problem((8, 8), 1)
    import torch
    a = torch.from_numpy(p.a).to("cuda")
    prob = mm.MMProblem()
    prob.d = 2
    prob.n[0], prob.n[1], prob.n[2] = 8, 8, 1
    prob.lam = 1.0
    prob.a = a.data_ptr()
    h = c_void_p()
    for bad in (1, 2, 8):
        st = mm.lib().mumode_setup(ctx.handle, byref(prob), 1e-3, mm.MM_LAWSON, 1, 0, mm.MM_SLICED, bad, byref(h))
        assert st == mm.MM_EINVAL
    with pytest.raises(ValueError):
        mm.prec_code("sliced8")
    # the ERK stacked contraction (q + 1) n = 32768 is too long for exact int32 level sums
    big = torch.zeros(4098 * 4098, dtype=torch.float64, device="cuda")
    prob.n[0], prob.n[1] = 4096, 4096
    prob.a = big.data_ptr()
    st = mm.lib().mumode_setup(ctx.handle, byref(prob), 1e-3, mm.MM_ERK, 0, 7, mm.MM_SLICED, 7, byref(h))
    assert st == mm.MM_EINVAL
    assert "too long" in ctx.error()


def test_server_sliced_request(mm):
    import time
    p = synth.smooth_problem((40, 36, 32), 50, tau=1e-3, steps=10)
    srv = mm.Server(0, max_active=4)
    try:
        rid = mm.solve_submit(srv, p, prec="sliced6")[1]
        t0 = time.time()
        while True:
            st, u, _ = mm.solve_poll(srv, rid, p.shape)
            if st != mm.MM_NOT_READY:
                break
            assert time.time() - t0 < 120
            time.sleep(0.001)
    finally:
        srv.close()
    assert st == mm.MM_OK
    ref = sliced.solve(p, 6)
    emax = max(float(np.max(np.abs(M))) for M in oracle_op(p).factors(1.0))
    assert np.max(np.abs(u - ref)) <= flip_bar(6, emax) * amplification(p) * float(np.max(np.abs(ref)))
