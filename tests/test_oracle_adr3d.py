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


def _kron_sum(mats):
    """The dense Kronecker sum A_d (+) ... (+) A_1 on C-ordered grid vectors (x1 fastest)."""
    K = np.zeros((1, 1))
    for A in reversed(mats):          # build from the slowest axis (the last) inwards
        K = np.kron(K, np.eye(A.shape[0])) + np.kron(np.eye(K.shape[0]), A)
    return K


@pytest.mark.parametrize("bc,beta_bar", [((1, 0, 1), (0.0, 0.6, 0.0)), ((1, 1), (1.5, -2.0)), ((0, 1, 1), (2.0, -1.0, 0.3))])
def test_exact_phi_against_augmented_exponentials(bc, beta_bar):
    """phi1 and phi2 of the Kronecker sum through the 1D eigenbases, against the exponential
    of the augmented matrices [[tau K, v, 0], [0, 0, 1], [0, 0, 0]], whose last column holds
    phi1(tau K) v and phi2(tau K) v (Saad 1992; Al-Mohy and Higham 2011), on small mixed
    Dirichlet/Neumann grids with advection in A."""
    import scipy.linalg
    n = (5, 4, 3)[: len(bc)]
    p = synth.smooth_problem(n, 12, tau=3e-3, beta_bar=beta_bar, q=0)
    p.bc = bc
    be = adr3d.Backend(p)
    K = _kron_sum(be.A)
    v = np.random.default_rng(13).standard_normal(p.shape)
    N = K.shape[0]
    M = np.zeros((N + 2, N + 2))
    M[:N, :N] = p.tau * K
    M[:N, N] = v.ravel()
    M[N, N + 1] = 1.0
    E = scipy.linalg.expm(M)
    ref1, ref2 = E[:N, N].reshape(p.shape), E[:N, N + 1].reshape(p.shape)
    from oracle import expo as X
    assert np.max(np.abs(be.funv(X.phi1, v) - ref1)) <= 1e-12 * np.max(np.abs(ref1))
    assert np.max(np.abs(be.phi1v(v) - ref1)) <= 1e-12 * np.max(np.abs(ref1))
    assert np.max(np.abs(be.phi2v(v) - ref2)) <= 1e-12 * np.max(np.abs(ref2))
    # the same identity through the all-Dirichlet oracle (a different code path) on a
    # Dirichlet grid, so that the augmented construction itself is checked
    pd = synth.smooth_problem(n, 12, tau=3e-3, beta_bar=beta_bar, q=0)
    op = X.KronOperator(pd.n, adr.extracted_amax(pd.a), pd.lam, pd.beta_bar, pd.tau)
    bd = adr3d.Backend(pd)
    assert np.max(np.abs(bd.phi2v(v) - op.phi2v_exact(v))) <= 1e-12 * np.max(np.abs(op.phi2v_exact(v)))


def test_exact_phi_schemes_converge_on_mixed_data():
    """EE (order 1) and erk2p2, ETD2RK with exact phi1 (order 2) on the Sec. 5.2 problem at
    N = 8 with the advection left in g (beta_bar = 0), against a small-step Lawson2b
    reference: observed orders within 0.2 of the classical ones."""
    def prob(scheme, m):
        p = synth.paper3d_problem(8, -1.0, 0.5, scheme=scheme, steps=m)
        p.beta_bar = (0.0, 0.0, 0.0)
        p.q = 0
        return p
    ref = adr3d.solve(prob("l2b", 2 ** 12))
    for sch, order in (("ee", 1), ("erk2p2", 2), ("etd2rk", 2)):
        e = [Sch.rel_inf_error(adr3d.solve(prob(sch, m)), ref) for m in (32, 64, 128)]
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(rates - order) < 0.2), (sch, e, rates)
