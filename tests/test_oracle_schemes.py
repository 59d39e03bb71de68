"""Pins for the oracle's time steps (Appendix) against Sec. 2 and an implicit reference."""
import numpy as np
import pytest

import synth
from oracle import schemes as S
from oracle import stability as St


def _mode_problem(n, ks, lam, tau, q=4):
    """a == 1, beta = 0, r = 0: g = (1 - lam) Lap_h u; u0 one discrete sine mode."""
    d = len(n)
    p = synth.constant_problem(n, 0, a_const=1.0, tau=tau, steps=1, lam=lam, q=q)
    vecs = [np.sin(ks[mu] * np.pi * np.arange(1, n[mu] + 1) / (n[mu] + 1)) for mu in range(d)]
    u0 = np.ones(1)
    for v in reversed(vecs):
        u0 = np.multiply.outer(u0, v)
    p.u0 = u0.reshape(tuple(reversed(n)))
    z = tau * sum(-4.0 * (n[mu] + 1) ** 2 * np.sin(ks[mu] * np.pi / (2 * (n[mu] + 1))) ** 2 for mu in range(d))
    return p, z


EXACT = ["ee", "le", "sle", "erk2p2", "erk2p1", "l2a", "l2b", "sl2", "etd2rk"]


@pytest.mark.parametrize("scheme", EXACT)
@pytest.mark.parametrize("lam", [1.0, 0.5, 0.35])
@pytest.mark.parametrize("ks", [(1, 2, 1), (5, 3, 7)])
def test_mode_amplification_is_phi(scheme, lam, ks):
    """one step multiplies a discrete sine mode by the paper's Phi(z, lam)."""
    p, z = _mode_problem((9, 8, 10), ks, lam, tau=1e-3)
    be = S.GridBackend(p, phi="exact")
    u1 = S.STEPS[scheme](p.u0, be, p.tau)
    ratio = St.PHI[scheme](np.array([z]), lam)[0]
    assert np.max(np.abs(u1 - ratio * p.u0)) <= 1e-13 * np.max(np.abs(p.u0)), (z, ratio)


@pytest.mark.parametrize("q", [4, 6])
@pytest.mark.parametrize("lam", [1.0, 0.6])
def test_mode_amplification_quadrature_forms(q, lam):
    p, z = _mode_problem((12, 11), (3, 5), lam, tau=4e-3, q=q)
    be = S.GridBackend(p, phi="quad")
    for scheme, phi in (("etd2rk", St.phi_etd2rk_quad), ("erk2p1f", St.phi_erk2p1f_quad)):
        u1 = S.STEPS[scheme](p.u0, be, p.tau)
        ratio = phi(np.array([z]), lam, q)[0]
        assert np.max(np.abs(u1 - ratio * p.u0)) <= 1e-13 * np.max(np.abs(p.u0)), scheme


@pytest.fixture(scope="module")
def radau_reference():
    """the same semi-discrete ODE solved by an implicit Radau IIA method (scipy)."""
    from scipy.integrate import solve_ivp
    from oracle import adr
    p = synth.smooth_problem((15, 14), 7, a_amp=0.9, beta=(4.0, -3.0), r=synth.R_CUBIC, tau=0.0,
                             steps=0)
    T = 0.02
    shape = p.u0.shape

    def rhs(t, y):
        return adr.full_rhs(y.reshape(shape), p.a, p.beta, p.r).ravel()

    sol = solve_ivp(rhs, (0.0, T), p.u0.ravel(), method="Radau", rtol=1e-12, atol=1e-13)
    return p, T, sol.y[:, -1].reshape(shape)


@pytest.mark.parametrize("scheme,order,phi", [("le", 1, "exact"), ("l2b", 2, "exact"),
                                              ("etd2rk", 2, "exact"), ("sle", 1, "exact"),
                                              ("l2a", 2, "exact"), ("sl2", 2, "exact"),
                                              ("ee", 1, "exact"), ("erk2p2", 2, "exact")])
def test_observed_order(radau_reference, scheme, order, phi):
    p, T, ref = radau_reference
    errs = []
    for m in (16, 32, 64):
        p.tau = T / m
        be = S.GridBackend(p, phi=phi)
        errs.append(S.rel_inf_error(S.integrate(p.u0, be, p.tau, m, scheme), ref))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert abs(slopes[-1] - order) < 0.15, (errs, slopes)
