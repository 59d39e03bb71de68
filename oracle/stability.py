"""Scalar stability functions Phi(z, lam) of Sec. 2 (oracle; test infrastructure only).

For the model problem u_t = lam Lap u + (1 - lam) Lap u, one Fourier (or
discrete sine) mode with Laplacian eigenvalue -k^2 is multiplied per step by
Phi(z, lam), z = -tau k^2. The formulas below are the ones stated in the proofs
of Theorems thm:expeuler, thm:lawsoneuler, thm:stabilizedlawsoneuler,
thm:exprk2phi2, thm:exprk2phi1, thm:lawson2ab and thm:stablawson2, and they are
written here independently of the step code in ``schemes`` so that one can pin
the other. The quadrature variants replace phi1(lam z) by
Q(lam z) = sum_j w_j exp(theta_j lam z).

Pins: test_oracle_stability (the lower bounds on lam of Table tab:stab).
"""
from __future__ import annotations

import numpy as np

from .expo import gauss_legendre_01, phi1, phi2


def phi_ee(z, lam):
    return 1.0 - 1.0 / lam + np.exp(z * lam) / lam


def phi_le(z, lam):
    return np.exp(lam * z) * (1.0 + (1.0 - lam) * z)


def phi_sle(z, lam):
    return 1.0 + z * np.exp(lam * z)


def phi_erk2p2(z, lam, c2=1.0):
    return 1.0 + z * phi1(lam * z) + z ** 2 * (1.0 - lam) * phi2(lam * z) * phi1(c2 * lam * z)


def phi_erk2p1(z, lam, c2=1.0):
    return 1.0 + z * phi1(lam * z) + 0.5 * z ** 2 * (1.0 - lam) * phi1(lam * z) * phi1(c2 * lam * z)


def phi_l2a(z, lam):
    return np.exp(lam * z) * (1.0 + z * (1.0 - lam) * (1.0 + z * (1.0 - lam) / 2.0))


def phi_l2b(z, lam):
    return np.exp(lam * z) * (1.0 + 0.5 * z * (1.0 - lam) + 0.5 * z * (1.0 - lam) * (1.0 + z * (1.0 - lam)))


def phi_sl2(z, lam, alpha=0.327):
    return 1.0 + z * np.exp(lam * z / 2.0) + 0.5 * z ** 2 * (1.0 - lam) * np.exp((1.0 + alpha) * lam * z)


PHI = {"ee": phi_ee, "le": phi_le, "sle": phi_sle, "erk2p2": phi_erk2p2, "erk2p1": phi_erk2p1,
       "l2a": phi_l2a, "l2b": phi_l2b, "sl2": phi_sl2, "etd2rk": phi_erk2p1}


def quad_phi1(x, q):
    """Q_q(x) = sum_j w_j exp(theta_j x), the Gauss-Legendre phi1 surrogate."""
    th, w = gauss_legendre_01(q)
    x = np.asarray(x, dtype=np.float64)
    return sum(wj * np.exp(tj * x) for tj, wj in zip(th, w))


def phi_etd2rk_quad(z, lam, q):
    """Amplification of the ETD2RK form with phi1 replaced by Q_q:
    U = e^{lam z} + (1-lam) z Q, u+ = U + (1-lam) z/2 Q (U - 1)."""
    Q = quad_phi1(lam * z, q)
    U = np.exp(lam * z) + (1.0 - lam) * z * Q
    return U + 0.5 * (1.0 - lam) * z * Q * (U - 1.0)


def phi_erk2p1f_quad(z, lam, q):
    """Amplification of the Appendix erk2p1 form with phi1 replaced by Q_q:
    U = 1 + z Q, u+ = U + (1-lam) z/2 Q (U - 1)."""
    Q = quad_phi1(lam * z, q)
    U = 1.0 + z * Q
    return U + 0.5 * (1.0 - lam) * z * Q * (U - 1.0)


def stability_bound(phi, lam_lo=0.05, lam_hi=1.0, zmin=-2000.0, npts=200001, tol=1e-6, **kw):
    """Smallest lam in [lam_lo, lam_hi] with max_{z in [zmin, 0]} |Phi(z, lam)| <= 1,
    by bisection over lam on a dense z grid (log-spaced toward -inf)."""
    z = -np.concatenate([np.linspace(0.0, 50.0, npts), np.geomspace(50.0, -zmin, 20001)])

    def ok(lam):
        return np.max(np.abs(phi(z, lam, **kw))) <= 1.0 + 1e-12

    lo, hi = lam_lo, lam_hi
    if not ok(hi):
        return None
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi
