"""Pins for the oracle's 1D factors, mu-mode action and phi1 (Sec. 1, Sec. 5.2)."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import brute, expo
from oracle.adr import operator_1d


@pytest.mark.parametrize("n,amax,lam,bb,ct", [(7, 1.9, 1.0, 0.0, 1e-3), (31, 1.3, 1.0, 0.0, 5e-4),
                                               (63, 1.5, 1.0, 0.0, 1e-3), (20, 1.0, 0.5, 3.0, 2e-3),
                                               (12, 2.0, 0.7, -5.0, 1e-2)])
def test_factor_vs_scipy_expm(n, amax, lam, bb, ct):
    """closed form through the sine transform vs Pade scaling-and-squaring (scipy)."""
    E = expo.exp_factor(n, amax, lam, bb, ct)
    R = expm(ct * operator_1d(n, amax, lam, bb))
    assert np.max(np.abs(E - R)) <= 1e-14 * max(1.0, np.max(np.abs(R))) * 10


def _nonsym_tridiag(rng, n):
    return (np.diag(rng.uniform(-3, -1, n)) + np.diag(rng.uniform(0.2, 1.5, n - 1), 1)
            + np.diag(rng.uniform(0.0, 0.8, n - 1), -1))


@pytest.mark.parametrize("sizes", [(5, 7), (7, 4), (5, 6, 7), (4, 3, 5), (8, 8, 8)])
def test_mumode_equals_expm_of_kron_sum(sizes):
    """exp(A_d (+) .. (+) A_1) vec(V) = vec(V x_1 e^{A_1} .. x_d e^{A_d}), nonsymmetric factors."""
    rng = np.random.default_rng(sum(sizes))
    mats = [_nonsym_tridiag(rng, n) for n in sizes]
    V = rng.standard_normal(tuple(reversed(sizes)))
    full = expm(brute.kron_sum(mats)) @ V.ravel()
    mm = expo.tucker(V, [expm(M) for M in mats]).ravel()
    assert np.max(np.abs(full - mm)) <= 1e-13 * np.max(np.abs(full))


def test_mumode_axis_order_matters():
    """a transposed operand or swapped axes would not pass the identity above."""
    rng = np.random.default_rng(5)
    mats = [_nonsym_tridiag(rng, n) for n in (5, 6, 7)]
    V = rng.standard_normal((7, 6, 5))
    full = expm(brute.kron_sum(mats)) @ V.ravel()
    wrong = expo.tucker(V, [expm(M).T for M in mats]).ravel()
    assert np.max(np.abs(full - wrong)) > 1e-3 * np.max(np.abs(full))


def test_kron_operator_expv_brute():
    p = synth.smooth_problem((6, 5, 4), 11, tau=2e-3, beta_bar=(1.0, -2.0, 0.5), lam=0.8)
    amax = float(p.a.max())
    op = expo.KronOperator(p.n, amax, p.lam, p.beta_bar, p.tau)
    mats = [operator_1d(p.n[mu], amax, p.lam, p.beta_bar[mu]) for mu in range(3)]
    K = brute.kron_sum(mats)
    for c in (1.0, 0.5, 0.2113):
        ref = expm(c * p.tau * K) @ p.u0.ravel()
        got = op.expv(c, p.u0).ravel()
        assert np.max(np.abs(ref - got)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("bb", [(0.0, 0.0), (2.0, -1.0)])
def test_phi1_exact_vs_augmented_matrix(bb):
    p = synth.smooth_problem((9, 7), 3, tau=5e-3, beta_bar=bb)
    amax = float(p.a.max())
    op = expo.KronOperator(p.n, amax, p.lam, p.beta_bar, p.tau)
    K = brute.kron_sum([operator_1d(p.n[mu], amax, p.lam, p.beta_bar[mu]) for mu in range(2)])
    ref = brute.augmented_phi1(K, p.u0.ravel(), p.tau)
    got = op.phi1v_exact(p.u0).ravel()
    assert np.max(np.abs(ref - got)) <= 1e-13 * np.max(np.abs(ref))


def test_phi2_exact_vs_augmented_matrix():
    """phi2(X) v is the top-right block of expm([[X, v, 0], [0, 0, 1], [0, 0, 0]])."""
    p = synth.smooth_problem((8, 6), 4, tau=5e-3)
    amax = float(p.a.max())
    op = expo.KronOperator(p.n, amax, p.lam, p.beta_bar, p.tau)
    K = brute.kron_sum([operator_1d(p.n[mu], amax, 1.0, 0.0) for mu in range(2)])
    N = K.shape[0]
    B2 = np.zeros((N + 2, N + 2))
    B2[:N, :N] = p.tau * K
    B2[:N, N] = p.u0.ravel()
    B2[N, N + 1] = 1.0
    ref2 = expm(B2)[:N, N + 1]
    got = op.phi2v_exact(p.u0).ravel()
    assert np.max(np.abs(ref2 - got)) <= 1e-13 * np.max(np.abs(ref2))


@pytest.mark.parametrize("q", [1, 2, 4, 6])
def test_gauss_legendre_nodes(q):
    th, w = expo.gauss_legendre_01(q)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all((th > 0) & (th < 1))
    for p_ in range(2 * q):
        assert abs(np.sum(w * th ** p_) - 1.0 / (p_ + 1)) < 5e-15
    assert abs(np.sum(w * th ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-9
    # symmetric about 1/2, so exp(theta) and exp(1 - theta) rules coincide
    assert np.allclose(np.sort(th), np.sort(1.0 - th), atol=1e-15)


def test_quadrature_phi1_matches_exact_on_smooth_data():
    """for |tau*lambda| <= ~1 the 4-node rule is accurate to 1e-9 (Gauss error term)."""
    p = synth.smooth_problem((15, 15), 1, tau=1e-5, u_kmax=3)
    amax = float(p.a.max())
    op = expo.KronOperator(p.n, amax, p.lam, p.beta_bar, p.tau)
    ex = op.phi1v_exact(p.u0)
    qd = op.phi1v_quad(p.u0, 4)
    assert np.max(np.abs(ex - qd)) <= 1e-9 * np.max(np.abs(ex))


@pytest.mark.parametrize("sizes", [(12, 10), (9, 8, 7)])
def test_sine_series_closed_form(sizes):
    """a == c, beta = 0, r = 0, lam = 1: g == 0, so LE and L2b reproduce
    u^m = sum_k c_k exp(m tau c sum_mu mu_k/h^2) prod sin(k_mu pi x_mu),
    mu_k = -4 sin^2(k pi h/2), exactly (semi-discrete closed form)."""
    from oracle import schemes as S
    kmax, seed, cval, m = 3, 17, 1.7, 6
    p = synth.constant_problem(sizes, seed, a_const=cval, u_kmax=kmax, tau=2e-3, steps=m)
    coef = synth.sine_coefficients(sizes, seed, kmax)
    d = len(sizes)
    hs = [1.0 / (n + 1) for n in sizes]
    xs = [np.arange(1, n + 1) * h for n, h in zip(sizes, hs)]
    ref = np.zeros(tuple(reversed(sizes)))
    for kk in np.ndindex(*coef.shape):          # kk = (k_d-1, .., k_1-1)
        ks = [kk[d - 1 - mu] + 1 for mu in range(d)]
        lam_k = sum(-4.0 * np.sin(ks[mu] * np.pi * hs[mu] / 2) ** 2 / hs[mu] ** 2 for mu in range(d))
        mode = np.ones(1)
        for mu in reversed(range(d)):
            mode = np.multiply.outer(mode, np.sin(ks[mu] * np.pi * xs[mu]))
        ref += coef[kk] * np.exp(m * p.tau * cval * lam_k) * mode.reshape(ref.shape)
    for scheme in ("le", "l2b"):
        u = S.solve(p, scheme=scheme)
        assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref)), scheme


def _expm_longdouble(M):
    """exp(M) in extended precision (numpy long double) by a Taylor series of M/2^s with
    |M/2^s|_1 <= 1/4, then s squarings: an independent method whose rounding (~1e-19 per
    operation, doubled by each squaring) is far below FP64's."""
    A = np.asarray(M, dtype=np.longdouble)
    nrm = float(np.max(np.sum(np.abs(A), axis=0)))
    s = max(0, int(np.ceil(np.log2(max(nrm, 1e-300) / 0.25))))
    B = A / np.longdouble(2.0) ** s
    X = np.eye(A.shape[0], dtype=np.longdouble)
    term = np.eye(A.shape[0], dtype=np.longdouble)
    for k in range(1, 30):
        term = term @ B / k
        X = X + term
    for _ in range(s):
        X = X @ X
    return X


@pytest.mark.slow
@pytest.mark.parametrize("n,amax,ct", [(255, 1.9, 5e-3), (127, 1.465, 5e-3)])
def test_stiff_factor_vs_extended_precision(n, amax, ct):
    """Stiff factors (|ct A|_1 up to 2.5e3): the closed form stays within a few units of
    FP64 rounding of an extended-precision scaling-and-squaring exponential. Evaluating
    the eigenvalues as delta + 2 sigma cos(theta) instead loses ~2 |delta ct| u to
    cancellation (1.4e-13 relative at the first size) and fails this bar."""
    E = expo.exp_factor(n, amax, 1.0, 0.0, ct)
    R = _expm_longdouble(ct * operator_1d(n, amax, 1.0, 0.0))
    err = float(np.max(np.abs(E - R)) / np.max(np.abs(R)))
    assert err <= 5e-15, err
