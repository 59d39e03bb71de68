"""Pins of oracle/adr3d.py (the problem of Sec. 5.2 with Dirichlet/Neumann data and the
non-divergence diffusion form) against facts that do not depend on it: the errors
printed in Figure fig:adr3d_diffl, textbook eigenpairs, an independent implementation
of the all-Dirichlet case, and consistency identities."""
import os

import numpy as np
import pytest

import synth
from oracle import adr, adr3d, expo
from oracle import schemes as Sch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig6_adr3d_lambda_errors.txt")


def printed_points():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        b, sch, lam, err = line.split()
        rows.append((float(b), sch, float(lam), float(err)))
    return rows


@pytest.fixture(scope="module")
def references():
    """The paper's reference: Lawson2b with a small step (here m = 2^14 at T = 1/4)."""
    return {b: adr3d.solve(synth.paper3d_problem(16, b, 1.0, scheme="l2b", steps=2 ** 14)) for b in (-0.01, -1.0)}


def test_fig6_printed_errors(references):
    """Every point of the four panels (LE, SLE, L2a, SL2; b = -0.01 and -1; N = 2^4,
    m = 2^8): relative infinity-norm error at T against the reference. The gaps are one
    constant per advection speed (3.3e-10 at b = -0.01, 2.2e-9 at b = -1), the size of the
    references' own error (2^14 against 2^15 steps: 6e-10 at b = -1), so the bar is that
    floor plus 1e-5 relative; the smallest printed errors are 6.5e-8."""
    rows = printed_points()
    assert len(rows) == 156
    for b, sch, lam, err in rows:
        u = adr3d.solve(synth.paper3d_problem(16, b, lam, scheme=sch))
        e = Sch.rel_inf_error(u, references[b])
        assert abs(e - err) <= 1e-5 * err + 3e-9, (b, sch, lam, e, err)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_dirichlet_neumann_second_difference_eigenpairs(n):
    """Centred second differences on x_i = i/n, zero value at 0 and the mirror ghost at 1:
    eigenvectors sin((2k-1) pi x / 2), eigenvalues -4 n^2 sin^2((2k-1) pi / (4n))."""
    A = adr3d.operator_1d(n, adr3d.NEUMANN, 1.0, 0.0)
    x = adr3d.nodes(n, adr3d.NEUMANN)
    for k in range(1, n + 1):
        v = np.sin((2 * k - 1) * np.pi * x / 2)
        mu = -4.0 * n * n * np.sin((2 * k - 1) * np.pi / (4 * n)) ** 2
        assert np.max(np.abs(A @ v - mu * v)) <= 1e-12 * abs(mu) * np.max(np.abs(v))


@pytest.mark.parametrize("n", [(7, 9), (6, 5, 8)])
def test_all_dirichlet_flux_form_matches_adr(n):
    p = synth.smooth_problem(n, 4, beta=(3.0, -2.0, 1.5)[: len(n)], lam=0.8, beta_bar=(1.0, 0.5, -0.25)[: len(n)],
                             r=(0.1, 0.7, -0.4, 0.2), tau=2e-3)
    amax = adr.extracted_amax(p.a)
    bcs = (0,) * p.d
    g1 = adr3d.remainder(p.u0, p.a, p.beta, p.r, p.lam, p.beta_bar, amax, bcs, "flux")
    g2 = adr.remainder(p.u0, p.a, p.beta, p.r, p.lam, p.beta_bar, amax)
    assert np.max(np.abs(g1 - g2)) <= 1e-12 * np.max(np.abs(g2))
    F1 = adr3d.full_rhs(p.u0, p.a, p.beta, p.r, bcs, "flux")
    F2 = adr.full_rhs(p.u0, p.a, p.beta, p.r)
    assert np.max(np.abs(F1 - F2)) <= 1e-12 * np.max(np.abs(F2))
    for mu in range(p.d):
        A1 = adr3d.operator_1d(p.n[mu], 0, p.lam * amax, p.beta_bar[mu])
        A2 = adr.operator_1d(p.n[mu], amax, p.lam, p.beta_bar[mu])
        assert np.max(np.abs(A1 - A2)) <= 1e-12 * np.max(np.abs(A2))
    # the exponential action: scipy expm of the dense matrices vs the sine-transform closed form
    be = adr3d.Backend(p)
    op = expo.KronOperator(p.n, amax, p.lam, p.beta_bar, p.tau)
    assert np.max(np.abs(be.expv(1.0, p.u0) - op.expv(1.0, p.u0))) <= 1e-13 * np.max(np.abs(p.u0))


@pytest.mark.parametrize("form", ["nondiv", "flux"])
@pytest.mark.parametrize("bc", [(1, 1, 1), (0, 1, 0), (1, 0)])
def test_full_rhs_is_extracted_operator_plus_remainder(bc, form):
    n = (9, 7, 6)[: len(bc)]
    p = synth.smooth_problem(n, 8, beta=(2.0, -1.0, 0.5)[: len(n)], lam=0.7, beta_bar=(1.5, 0.25, -0.5)[: len(n)],
                             r=(0.0, 1.0, 0.0, 1.0))
    p.bc, p.form = bc, form
    be = adr3d.Backend(p)
    u = np.random.default_rng(3).standard_normal(p.shape)
    Au = sum(expo.mode_product(u, A, mu) for mu, A in enumerate(be.A))
    F = be.F(u)
    assert np.max(np.abs(F - (Au + be.g(u)))) <= 1e-12 * np.max(np.abs(F))


def test_neumann_laplacian_second_order():
    """Lap of sin(pi x1/2) sin(pi x2/2) sin(pi x3/2) (zero at 0, zero normal derivative at
    1) is -3 pi^2/4 times the field; the discrete error falls by 4 per halving of h."""
    errs = []
    for N in (8, 16, 32):
        x = adr3d.nodes(N, adr3d.NEUMANN)
        s = np.sin(np.pi * x / 2)
        u = s[:, None, None] * s[None, :, None] * s[None, None, :]
        a = np.ones((N + 2,) * 3)
        lap = adr3d.full_rhs(u, a, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0), (1, 1, 1), "nondiv")
        errs.append(np.max(np.abs(lap + 0.75 * np.pi ** 2 * u)))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs
