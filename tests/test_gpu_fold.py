"""Folded FP64 mode products against the plain products and the oracle.

On an axis with zero Dirichlet data at both ends and no advection moved into A, the
extracted 1D operator is a symmetric Toeplitz matrix and every factor exp(c tau A_mu) is
centrosymmetric; the folded kernels form the sums and differences of mirrored grid entries
and multiply them by two half-size factors. They must agree with the plain products to
rounding and with the oracle within the FP64 bar, for odd and even axis lengths (a middle
point or none), 2D and 3D grids, the padded stage layouts of the Lawson steps, in-place
actions, quadrature factors and the ERK steps, and must leave axes without the symmetry
(advection in A, a zero normal derivative) to the plain product.
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo
from oracle import schemes as Sch

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
    c.set_fold(1)
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


def expv(mm, ctx, p, V, mode, j=0, in_place=False):
    ctx.set_fold(mode)
    op = mm.setup_problem(ctx, p)
    x = dev(V)
    out = x if in_place else dev(np.zeros(p.shape))
    mm.mumode_expv(op, x, out, j=j)
    got = host(out)
    op.close()
    return got


@pytest.mark.parametrize("n", [(1, 1), (2, 3), (9, 13), (64, 63), (1, 1, 1), (2, 2, 2), (5, 6, 7), (8, 9, 10),
                               (17, 33, 9), (130, 129, 127)])
def test_folded_exp_action(mm, ctx, n):
    p = synth.smooth_problem(n, 31, tau=1e-3)
    V = np.random.default_rng(32).standard_normal(p.shape)
    plain = expv(mm, ctx, p, V, 0)
    folded = expv(mm, ctx, p, V, 2)
    ref = oracle_op(p).expv(1.0, V)
    assert relerr(plain, ref) <= FP64_TOL
    assert relerr(folded, ref) <= FP64_TOL
    assert relerr(folded, plain) <= 1e-13


def test_folded_in_place_and_quadrature_factor(mm, ctx):
    """in place (the folded kernel reads mirrored entries of its input: the action writes
    through intermediates, so the last product may overwrite the input) and exp factor j =
    2 of an ERK operator (a quadrature node), both folded."""
    p = synth.smooth_problem((66, 41, 35), 33, tau=2e-3, scheme="etd2rk", q=4)
    V = np.random.default_rng(34).standard_normal(p.shape)
    got = expv(mm, ctx, p, V, 2, in_place=True)
    assert relerr(got, oracle_op(p).expv(1.0, V)) <= FP64_TOL
    th, _ = expo.gauss_legendre_01(4)
    got2 = expv(mm, ctx, p, V, 2, j=2)
    assert relerr(got2, oracle_op(p).expv(th[1], V)) <= FP64_TOL


@pytest.mark.parametrize("n,q", [((12, 11), 4), ((16, 9, 13), 4), ((20, 18, 21), 6)])
def test_folded_stacked_phi1(mm, ctx, n, q):
    """The quadrature φ1 action: its last mode contracts the stacked weighted factors
    [w_j E(θ_j)], which fold block by block (odd and even last axes, two and three dims)."""
    p = synth.smooth_problem(n, 38, tau=2e-3, scheme="etd2rk", q=q)
    ctx.set_fold(2)
    op = mm.setup_problem(ctx, p)
    V = np.random.default_rng(39).standard_normal(p.shape)
    out = dev(np.zeros(p.shape))
    mm.mumode_phi1v(op, dev(V), out)
    got = host(out)
    op.close()
    assert relerr(got, oracle_op(p).phi1v_quad(V, q)) <= FP64_TOL


def test_axes_without_symmetry_stay_plain(mm, ctx):
    """advection in A (nonsymmetric factors) on some axes: with fold = 2 those axes keep
    the plain product (a folded product of a nonsymmetric factor would miss the oracle by
    far more than the bar) and the symmetric axis folds."""
    p = synth.smooth_problem((21, 18, 15), 35, tau=2e-3, beta_bar=(4.0, 0.0, -3.0), lam=0.9)
    V = np.random.default_rng(36).standard_normal(p.shape)
    got = expv(mm, ctx, p, V, 2)
    assert relerr(got, oracle_op(p).expv(1.0, V)) <= FP64_TOL


STEPS = [("l2b", (20, 17, 23), 6, 1e-3), ("le", (33, 31, 29), 6, 1e-3), ("l2b", (64, 63), 10, 1e-3),
         ("etd2rk", (19, 22, 17), 4, 2e-3), ("erk2p1f", (18, 21, 16), 4, 2e-3), ("l2b", (129, 130, 131), 2, 5e-4)]


@pytest.mark.parametrize("scheme,n,steps,tau", STEPS, ids=[f"{c[0]}-{'x'.join(map(str, c[1]))}" for c in STEPS])
def test_folded_steps_match_oracle(mm, ctx, scheme, n, steps, tau):
    p = synth.smooth_problem(n, 37, tau=tau, steps=steps, scheme=scheme, q=4)
    ctx.set_fold(2)
    op = mm.setup_problem(ctx, p)
    u = dev(p.u0)
    mm.step(op, u, p.steps)
    status = mm.mm_check(op)
    got = host(u)
    op.close()
    assert status == mm.MM_OK
    assert relerr(got, Sch.solve(p)) <= FP64_TOL


def test_fold_full_size_default(mm, ctx):
    """255^3 Lawson2b, two steps, default mode (folded at this size) against the plain
    products: the same solution within the FP64 bar (the two round differently in each of
    the six 255-term products of a step; measured 2e-13). The element-wise comparison with
    the oracle at this size is the full-size step test of the parity suite, which runs
    folded by default."""
    p = synth.workload("3d_n255_l2b")
    res = {}
    for mode in (0, 1):
        ctx.set_fold(mode)
        op = mm.setup_problem(ctx, p)
        u = dev(p.u0)
        mm.lawson_step(op, u, 2)
        assert mm.mm_check(op) == mm.MM_OK
        res[mode] = host(u)
        op.close()
    assert relerr(res[1], res[0]) <= FP64_TOL


def test_fold_mode_validation(mm, ctx):
    with pytest.raises(mm.MumodeError):
        ctx.set_fold(3)
    with pytest.raises(mm.MumodeError):
        ctx.set_fold(-1)
