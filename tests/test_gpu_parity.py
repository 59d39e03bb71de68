"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar (FP64): max |gpu - oracle| <= 1e-12 * max |oracle| on every element. The GPU
factors come from Pade scaling-and-squaring and the oracle's from the sine-transform
closed form, so the two sides share no arithmetic; both are FP64, and 1e-12 leaves
room for the different rounding order of the contractions (a K = 255 FP64 dot
product carries about 255 * 1.1e-16 relative error) and of the Pade squarings.
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo
from oracle import schemes as S

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


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


def oracle_op(p):
    return expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau)


# ------------------------------------------------------------------ factors (Pade)
@pytest.mark.parametrize("n,scheme,tau", [((63, 63), "le", 1e-3), ((31, 20, 9), "etd2rk", 2e-3),
                                          ((127, 127, 127), "l2b", 5e-4), ((255, 255, 255), "l2b", 1e-3),
                                          ((383, 383, 383), "etd2rk", 2e-3)])
def test_factors_match_closed_form(mm, ctx, n, scheme, tau):
    if len(n) == 3 and n[0] == 383:
        p = synth.anisotropic_problem(383, 0, tau=tau, steps=1)
    else:
        p = synth.smooth_problem(n, 1, tau=tau, scheme=scheme, q=6 if scheme == "etd2rk" else 4)
    op = mm.setup_problem(ctx, p)
    amax, _ = op.info()
    assert amax == float(p.a.max())
    ref_op = oracle_op(p)
    th, _ = expo.gauss_legendre_01(p.q)
    cs = [1.0] + (list(th) if op.q else [])
    for mu in range(p.d):
        for j, c in enumerate(cs):
            E = op.factor(mu, j)
            R = ref_op.factors(c)[mu]
            # scaling-and-squaring loses ~2^s eps; at 383 (s = 9) the gap is 4.5e-13
            assert np.max(np.abs(E - R)) <= FP64_TOL * np.max(np.abs(R)), (mu, j)
    op.close()


# ------------------------------------------------------------------ stencil
# The kernel gives each lane P = 1, 2 or 4 consecutive x1 points (the P that pads n1 least
# to 64 P-point segments) and splits longer rows into segments whose ends are loaded
# separately: the cases cover every P, partly and exactly filled segments, and rows of
# several segments for each P (129, 257, 300: P = 1; 383: P = 2; 511: P = 4).
STENCIL_CASES = [(1, 1), (5, 7), (63, 63), (65, 9), (300, 7), (511, 5), (1, 1, 1), (5, 6, 7), (70, 9, 33),
                 (127, 127, 127), (129, 5, 6), (256, 4, 3), (257, 3, 4), (383, 6, 5)]


@pytest.mark.parametrize("n", STENCIL_CASES)
def test_remainder_and_full_rhs(mm, ctx, n):
    p = synth.smooth_problem(n, 2, beta=(3.0, -2.0, 1.5)[: len(n)], lam=0.8,
                             beta_bar=(1.0, 0.5, -0.25)[: len(n)], r=(0.1, 0.7, -0.4, 0.2))
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    import torch
    g = torch.empty_like(u)
    F = torch.empty_like(u)
    mm.remainder_eval(op, u, g, F)
    amax = adr.extracted_amax(p.a)
    gref = adr.remainder(p.u0, p.a, p.beta, p.r, p.lam, p.beta_bar, amax)
    Fref = adr.full_rhs(p.u0, p.a, p.beta, p.r)
    assert relerr(host(g), gref) <= 1e-13
    assert relerr(host(F), Fref) <= 1e-13
    op.close()


# ------------------------------------------------------------------ exp action
@pytest.mark.parametrize("n", [(1, 1), (9, 13), (63, 63), (200, 130), (1, 1, 1), (5, 6, 7), (17, 33, 9),
                               (130, 129, 127), (255, 255, 255)])
def test_exp_action(mm, ctx, n):
    p = synth.smooth_problem(n, 3, tau=1e-3)
    rng = np.random.default_rng(7)
    V = rng.standard_normal(p.shape)
    op = mm.setup_problem(ctx, p)
    out = dev(np.zeros(p.shape))
    mm.mumode_expv(op, dev(V), out)
    got = host(out)
    op.close()
    ref = oracle_op(p).expv(1.0, V)
    assert relerr(got, ref) <= FP64_TOL


def test_exp_action_in_place_and_nonsymmetric_factor(mm, ctx):
    """beta_bar != 0 makes the 1D factors nonsymmetric: a transposed factor fails here."""
    p = synth.smooth_problem((21, 18, 15), 4, tau=2e-3, beta_bar=(4.0, -3.0, 2.0), lam=0.9)
    op = mm.setup_problem(ctx, p)
    V = np.random.default_rng(8).standard_normal(p.shape)
    x = dev(V)
    mm.mumode_expv(op, x, x)
    ref = oracle_op(p).expv(1.0, V)
    assert relerr(host(x), ref) <= FP64_TOL
    op.close()


@pytest.mark.parametrize("n,q", [((12, 11), 4), ((16, 9, 13), 4), ((64, 63, 65), 6), ((127, 127, 127), 4)])
def test_phi1_quadrature_action(mm, ctx, n, q):
    p = synth.smooth_problem(n, 5, tau=2e-3, scheme="etd2rk", q=q)
    op = mm.setup_problem(ctx, p)
    V = np.random.default_rng(9).standard_normal(p.shape)
    out = dev(np.zeros(p.shape))
    mm.mumode_phi1v(op, dev(V), out)
    ref = oracle_op(p).phi1v_quad(V, q)
    assert relerr(host(out), ref) <= FP64_TOL
    # the quadrature nodes as factors: j-th exp action
    th, _ = expo.gauss_legendre_01(q)
    out2 = dev(np.zeros(p.shape))
    mm.mumode_expv(op, dev(V), out2, j=2)
    assert relerr(host(out2), oracle_op(p).expv(th[1], V)) <= FP64_TOL
    op.close()


# ------------------------------------------------------------------ whole steps
CASES = [
    ("le", (63, 63), 100, 1e-3),       # the 2D 63^2 Lawson-Euler workload, all 100 steps
    ("l2b", (63, 63), 20, 1e-3),
    ("l2b", (20, 17, 23), 10, 1e-3),
    ("le", (33, 31, 29), 10, 1e-3),
    ("etd2rk", (19, 22, 17), 6, 2e-3),
    ("erk2p1f", (19, 22, 17), 6, 2e-3),
    ("etd2rk", (40, 35), 10, 2e-3),
    ("l2b", (129, 130, 131), 3, 5e-4),
    ("l2b", (300, 40), 5, 1e-4),        # two-segment stencil rows
    ("etd2rk", (260, 9, 11), 3, 1e-4),
]


@pytest.mark.parametrize("scheme,n,steps,tau", CASES, ids=[f"{c[0]}-{'x'.join(map(str, c[1]))}" for c in CASES])
def test_steps_match_oracle(mm, ctx, scheme, n, steps, tau):
    if n == (63, 63) and scheme == "le":
        p = synth.workload("2d_n63_le")
    else:
        p = synth.smooth_problem(n, 6, tau=tau, steps=steps, scheme=scheme, q=4)
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    status = mm.mm_check(op)
    got = host(u)
    op.close()
    assert status == mm.MM_OK
    ref = S.solve(p)
    assert relerr(got, ref) <= FP64_TOL


def test_steps_compose(mm, ctx):
    """two calls of k steps equal one call of 2k steps, bit for bit (checkpoint/resume)."""
    p = synth.smooth_problem((24, 20, 16), 7, tau=1e-3, steps=8, scheme="l2b")
    op = mm.setup_problem(ctx, p)
    u1 = dev(p.u0)
    mm.step(op, u1, 8)
    u2 = dev(p.u0)
    mm.step(op, u2, 5)
    mm.step(op, u2, 3)
    assert np.array_equal(host(u1), host(u2))
    op.close()


# ------------------------------------------------------------------ full-size, one step
@pytest.mark.parametrize("name", ["3d_n255_l2b", "3d_n127_etd2rk", "3d_n127_l2b"])
def test_full_size_one_step(mm, ctx, name):
    """one step at the workload's full size and launch configuration, every element."""
    p = synth.workload(name)
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    mm.step(op, u, 1)
    status = mm.mm_check(op)
    got = host(u)
    op.close()
    assert status == mm.MM_OK
    ref = S.solve(p, steps=1)
    assert relerr(got, ref) <= FP64_TOL


# ------------------------------------------------------------------ errors and flags
def test_invalid_arguments(mm, ctx):
    p = synth.smooth_problem((8, 8), 1)
    a = dev(p.a)
    with pytest.raises(mm.MumodeError) as e:
        mm.mumode_setup(ctx, 4, (8, 8, 8), a, (0, 0, 0), (0, 0, 0, 0), 1e-3)
    assert e.value.status == mm.MM_EINVAL
    with pytest.raises(mm.MumodeError):
        mm.mumode_setup(ctx, 2, (8, 8), a, (0, 0), (0, 0, 0, 0), -1.0)
    with pytest.raises(mm.MumodeError):
        mm.mumode_setup(ctx, 2, (0, 8), a, (0, 0), (0, 0, 0, 0), 1e-3)
    op = mm.setup_problem(ctx, p)
    with pytest.raises(mm.MumodeError):
        mm.erk_step(op, dev(p.u0), 1)            # Lawson operator
    with pytest.raises(mm.MumodeError):
        mm.mumode_phi1v(op, dev(p.u0), dev(p.u0))
    op.close()


def test_nonfinite_state_is_flagged(mm, ctx):
    p = synth.smooth_problem((16, 15, 14), 1, tau=1e-3, scheme="l2b")
    op = mm.setup_problem(ctx, p)
    u0 = p.u0.copy()
    u0[3, 4, 5] = np.nan
    u = dev(u0)
    mm.step(op, u, 2)
    assert mm.mm_check(op) == mm.MM_EUNSTABLE
    op.close()
