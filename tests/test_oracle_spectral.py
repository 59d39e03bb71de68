"""Pins of oracle/spectral.py (periodic pseudo-spectral problems of Sec. 4 and 5.1)
against facts that do not depend on it: closed-form derivatives and exponentials of
trigonometric polynomials, the independent one-dimensional Fourier backend that
reproduces Figure fig:ad1dex0_diffdeltaa, the errors printed in Figure
fig:ad1dpx91_diffdelta, and the errors of Figure fig:adr2d_diffl with the lambda values of
Table tab:adr2d_lambdaopt."""
import os

import numpy as np
import pytest

import synth
from oracle import fourier1d as F1
from oracle import schemes as Sch
from oracle import spectral

PERIODIC = synth.PERIODIC


def _box(n, L, lam=0.7, beta_bar=None, form="flux", a_const=None):
    d = len(n)
    xs = [spectral.grid(n[mu], L[mu], -0.3 * mu) for mu in range(d)]
    mesh = np.meshgrid(*[xs[mu] for mu in reversed(range(d))], indexing="ij")
    X = list(reversed(mesh))
    a = np.stack([np.full(X[0].shape, a_const[mu]) for mu in range(d)]) if a_const else \
        np.stack([1.0 + 0.3 * np.sin(2 * np.pi / L[mu] * X[mu]) ** 2 for mu in range(d)])
    p = synth.Problem(d=d, n=tuple(n), a=a, u0=np.zeros(X[0].shape), beta=(0.0,) * d, r=(0.0,) * 4, tau=0.01,
                      steps=1, lam=lam, beta_bar=beta_bar or (0.0,) * d, bc=(PERIODIC,) * d, form=form,
                      length=tuple(L), velocity=None)
    return p, X


@pytest.mark.parametrize("n", [(16, 12), (15, 9, 8)])
def test_derivatives_of_trigonometric_polynomials(n):
    """d_mu and d_mumu of sin(k kappa x_mu + phase) for every |k| below the Nyquist
    wavenumber are k kappa cos(.) and -(k kappa)^2 sin(.) at the grid points."""
    L = (2 * np.pi, 3.0, 5.0)[: len(n)]
    p, X = _box(n, L)
    be = spectral.Spectral(p)
    for mu in range(len(n)):
        kap = 2 * np.pi / L[mu]
        for k in range(0, (n[mu] - 1) // 2 + 1):
            arg = k * kap * X[mu] + 0.4
            v = np.sin(arg)
            assert np.max(np.abs(be.d1(v, mu) - k * kap * np.cos(arg))) <= 1e-12 * max(1.0, k * kap) * n[mu]
            assert np.max(np.abs(be.d2(v, mu) + (k * kap) ** 2 * v)) <= 1e-12 * max(1.0, k * kap) ** 2 * n[mu]


def test_nyquist_convention():
    """For even n the Nyquist mode (-1)^j has zero first derivative and second derivative
    -(pi n / L)^2 (-1)^j."""
    p, X = _box((8, 6), (2.0, 3.0))
    be = spectral.Spectral(p)
    v = np.cos(np.pi * np.arange(8))[None, :] * np.ones((6, 1))
    assert np.max(np.abs(be.d1(v, 0))) <= 1e-13
    assert np.max(np.abs(be.d2(v, 0) + (np.pi * 8 / 2.0) ** 2 * v)) <= 1e-10


def test_exponential_of_a_mode_is_damped_translation():
    """A = lam a_max d_xx + beta_bar d_x: exp(tau A) cos(kappa x) = exp(-tau lam a_max kappa^2)
    cos(kappa (x + tau beta_bar)) (the advection generates a shift)."""
    n, L = (32, 4), (2 * np.pi, 1.0)
    p, X = _box(n, L, lam=0.6, beta_bar=(0.7, 0.0), a_const=(1.5, 1.0))
    be = spectral.Spectral(p)
    for k in (1, 3, 7):
        v = np.cos(k * X[0])
        want = np.exp(-p.tau * 0.6 * 1.5 * k * k) * np.cos(k * (X[0] + p.tau * 0.7))
        assert np.max(np.abs(be.expv(1.0, v) - want)) <= 1e-13
        # phi1 of the pure decay (beta_bar = 0 axis): (e^z - 1)/z on the mode
    p2, X2 = _box(n, L, lam=0.6, a_const=(1.5, 1.0))
    be2 = spectral.Spectral(p2, phi="exact")
    z = -p2.tau * 0.6 * 1.5 * 9
    assert np.max(np.abs(be2.phi1v(np.cos(3 * X2[0])) - np.expm1(z) / z * np.cos(3 * X2[0]))) <= 1e-13


def test_constant_coefficient_remainder():
    """With constant a and no velocity, g(sin kx) = (a - lam a_max) (-k^2) sin kx + r = -(1 -
    lam) a k^2 sin kx in both diffusion forms."""
    for form in ("flux", "nondiv"):
        p, X = _box((24, 5), (2 * np.pi, 2 * np.pi), lam=0.3, form=form, a_const=(2.0, 0.5))
        be = spectral.Spectral(p)
        v = np.sin(4 * X[0]) * np.cos(2 * X[1])
        want = (-(2.0 - 0.3 * 2.0) * 16 - (0.5 - 0.3 * 0.5) * 4) * v
        assert np.max(np.abs(be.g(v) - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("lam,scheme,m", [(1.0, "sle", 16), (0.5, "le", 64), (0.5, "l2b", 16), (1.0, "sl2", 64)])
def test_linear_1d_matches_the_fourier_backend(lam, scheme, m):
    """Sec. 4.1 (u_t = a u_xx, N = 2^12) through this backend against oracle/fourier1d.py,
    which reproduces the printed errors of Figure fig:ad1dex0_diffdeltaa."""
    p = synth.paper1d_problem(4096, lam, nonlinear=False, scheme=scheme, steps=m)
    u = spectral.solve(p)
    v = Sch.integrate(p.u0[0], F1.Fourier1D(4096, lam, p.tau), p.tau, m, scheme)
    assert np.max(np.abs(u[0] - v)) <= 1e-10 * np.max(np.abs(v))


# Figure fig:ad1dpx91_diffdelta (Sec. 4.2): N = 2^10, T = 1/10, m = 2^12 (scheme, lambda, error)
FIG_PX91 = [("sle", 1.0, 1.26214156559945e-4), ("sle", 0.5, 5.70882140624806e-05), ("sle", 0.183, 1.35086205056413e-05),
            ("le", 1.0, 4.84133061045172e-3), ("le", 0.218, 2.57438011667187e-4),
            ("ee", 1.0, 5.7047227927228e-05), ("l2b", 1.0, 3.69142379078708e-05), ("l2b", 0.301, 6.25505479242713e-07),
            ("l2a", 0.5, 4.78117833428809e-06), ("sl2", 1.0, 4.86274401250389e-07),
            ("sl2", 0.183, 8.10631356900742e-09), ("erk2p2", 1.0, 2.18171665233022e-07)]


def test_fig_px91_printed_errors():
    """Sec. 4.2: u_t = (a u_x)_x + u(1 - u), the reference being ERK2 with phi2 on the
    unsplit equation (the whole linear operator d_x a d_x exact through its
    eigendecomposition, 2^13 steps, self-converged to 1e-10): every listed point of the
    figure within 5e-4 relative (1e-3 for the two smallest errors, where the reference's
    own error shows)."""
    N, T = 1024, 0.1
    p = synth.paper1d_problem(N, 1.0, nonlinear=True, scheme="l2b", steps=4096)
    be = spectral.Spectral(p)
    eye = np.eye(N)
    D1 = np.stack([be.d1(eye[j][None, :], 0)[0] for j in range(N)], axis=1)
    Afull = D1 @ np.diag(p.a[0][0]) @ D1
    w, V = np.linalg.eigh(0.5 * (Afull + Afull.T))

    class Unsplit:
        def __init__(self, tau):
            self.tau = tau

        def _f(self, f, v):
            return (V @ (f * (V.T @ v[0])))[None, :]

        def phi1v(self, v):
            return self._f(spectral.phi_complex(1, self.tau * w).real, v)

        def phi2v(self, v):
            return self._f(spectral.phi_complex(2, self.tau * w).real, v)

        def g(self, v):
            return v * (1.0 - v)

        def F(self, v):
            return (Afull @ v[0])[None, :] + self.g(v)

    m = 2 ** 13
    ref = Sch.integrate(p.u0, Unsplit(T / m), T / m, m, "erk2p2")
    for sch, lam, err in FIG_PX91:
        q = synth.paper1d_problem(N, lam, nonlinear=True, scheme=sch, steps=4096)
        e = Sch.rel_inf_error(spectral.solve(q, phi="exact"), ref)
        tol = 1e-3 if err < 1e-7 else 5e-4
        assert abs(e - err) <= tol * err, (sch, lam, e, err)


def _fig_adr2d(N):
    path = os.path.join(os.path.dirname(__file__), "golden", "fig_adr2d_lambda_errors.txt")
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        n, sch, lam, err = line.split()
        if int(n) == N:
            rows.append((sch, float(lam), float(err)))
    return rows


def test_fig_adr2d_printed_errors_and_lambda_table():
    """Sec. 5.1 at N = 2^6, m = 2^8, T = 4 against a Lawson2b reference (lambda = 1, 2^13
    steps): the printed errors of LE, SLE, SL2 and EE within -2.5%/+1.5% (they come out
    about 2% low at most lambda, uniformly for EE: a systematic offset whose cause is not
    identified), L2a within -6%/+17%, and the smallest error on the printed lambda grid at
    the value of Table tab:adr2d_lambdaopt for LE (0.22), SLE (0.23), SL2 (0.57) and EE (0.50)."""
    ref = spectral.solve(synth.paper2d_problem(64, 1.0, scheme="l2b", steps=2 ** 13))
    table = {"le": 0.22, "sle": 0.23, "sl2": 0.57, "ee": 0.50, "l2a": None}
    rows = _fig_adr2d(64)
    for sch, lam_opt in table.items():
        pts = [(lam, err) for s, lam, err in rows if s == sch]
        assert len(pts) >= 13
        lo, hi = (0.975, 1.015) if sch != "l2a" else (0.94, 1.17)
        errs = []
        for lam, err in pts:
            e = Sch.rel_inf_error(spectral.solve(synth.paper2d_problem(64, lam, scheme=sch), phi="exact"), ref)
            assert lo * err <= e <= hi * err, (sch, lam, e, err)
            errs.append(e)
        if lam_opt is not None:
            assert abs(pts[int(np.argmin(errs))][0] - lam_opt) < 0.01, sch


@pytest.mark.parametrize("form", ["flux", "nondiv"])
def test_variable_coefficient_remainder_closed_form(form):
    """The remainder and F of the problem of Sec. 5.1 with its own diffusion tensor and
    velocity field (trigonometric polynomials) on u = sin(2 x1) cos(x2), against the
    derivatives written out by hand (product rule):
      d1(a11 d1 u) = (d1 a11)(d1 u) + a11 d11 u, div(b u) = sum (d_mu b_mu) u + b_mu d_mu u,
      A u = lam (a11^max d11 u + a22^max d22 u) + beta_bar . grad u, g = F - A u.
    Every product is band-limited well below the Nyquist wavenumber of N = 64, so the
    pseudo-spectral values are exact to rounding; a sign or a form error in either term
    (a d_mumu u for the flux form, -div(b u), beta_bar added instead of subtracted)
    misses by O(1)."""
    lam = 0.5
    p = synth.paper2d_problem(64, lam, scheme="l2b")
    p.form = form
    L = p.length[0]
    x = -3.0 * np.pi + L / 64 * np.arange(64)
    X2, X1 = np.meshgrid(x, x, indexing="ij")
    s1, c1, s2, c2 = np.sin(X1), np.cos(X1), np.sin(X2), np.cos(X2)
    u = np.sin(2 * X1) * c2
    u1, u11 = 2 * np.cos(2 * X1) * c2, -4 * np.sin(2 * X1) * c2
    u2, u22 = -np.sin(2 * X1) * s2, -np.sin(2 * X1) * c2
    a11, a22 = 0.5 + s1 ** 2 * s2 ** 2 / 6, 0.5 + c1 ** 2 * c2 ** 2 / 6
    a11_1, a22_2 = np.sin(2 * X1) * s2 ** 2 / 6, -(c1 ** 2) * np.sin(2 * X2) / 6
    b1, b2 = s1 ** 2 / 5, s2 ** 2 / 5
    b1_1, b2_2 = np.sin(2 * X1) / 5, np.sin(2 * X2) / 5
    amax = (float(p.a[0].max()), float(p.a[1].max()))
    react = p.r[0] + u * (p.r[1] + u * (p.r[2] + u * p.r[3]))
    adv = b1_1 * u + b1 * u1 + b2_2 * u + b2 * u2
    if form == "flux":
        diff = a11_1 * u1 + a11 * u11 + a22_2 * u2 + a22 * u22
    else:
        diff = a11 * u11 + a22 * u22
    F = diff + adv + react
    Au = lam * (amax[0] * u11 + amax[1] * u22) + p.beta_bar[0] * u1 + p.beta_bar[1] * u2
    be = spectral.Spectral(p)
    scale = float(np.max(np.abs(F)))
    assert np.max(np.abs(be.F(u) - F)) <= 1e-12 * scale
    assert np.max(np.abs(be.g(u) - (F - Au))) <= 1e-12 * scale
    assert np.max(np.abs(be.A(u) - Au)) <= 1e-12 * scale
