"""Lawson and exponential Runge-Kutta steps (oracle; test infrastructure only).

The Appendix lists the integrators for u' = A u + g(u) = F(u) (autonomous
problems here, so the time argument of g is dropped). Each step below is
written against a small backend with

    expv(c, v)  = exp(c tau A) v          phi1v(v) = phi1(tau A) v
    g(v)        = remainder               phi2v(v) = phi2(tau A) v
    F(v)        = full right-hand side

so that the same step code runs on the finite-difference grids (KronOperator)
and on the periodic Fourier setting used to reproduce Figure
fig:ad1dex0_diffdeltaa. c2 = 1 throughout for the ERK schemes (as in the
paper's experiments), alpha = 0.327 for the stabilized Lawson2 scheme
(Theorem thm:stablawson2).

ETD2RK (reading; the name is not the paper's): the second-order ERK with phi1
only, c2 = 1, written in the equivalent form that applies the exponential to u:
    U = e^{tau A} u + tau phi1(tau A) g(u),
    u+ = U + tau/2 phi1(tau A) (g(U) - g(u)).
With exact phi1 this is the Appendix scheme exactly (e^z = 1 + z phi1(z));
with quadrature phi1 it is the form used by the product path.

Pins: test_oracle_schemes (per-mode amplification equals the stability
functions of Sec. 2 for every scheme; observed orders vs an implicit reference)
and test_oracle_fig1 (printed errors of Sec. 4.1).
"""
from __future__ import annotations

from typing import Callable, Dict

import numpy as np

ALPHA_SL2 = 0.327


def step_le(u, be, tau):
    """Lawson-Euler: u+ = e^{tau A}(u + tau g(u))."""
    return be.expv(1.0, u + tau * be.g(u))


def step_sle(u, be, tau):
    """stabilized Lawson-Euler: u+ = u + tau e^{tau A} F(u)."""
    return u + tau * be.expv(1.0, be.F(u))


def step_l2a(u, be, tau):
    """Lawson2a: U = e^{tau/2 A}(u + tau/2 g(u)); u+ = e^{tau A} u + tau e^{tau/2 A} g(U)."""
    U = be.expv(0.5, u + 0.5 * tau * be.g(u))
    return be.expv(1.0, u) + tau * be.expv(0.5, be.g(U))


def step_l2b(u, be, tau):
    """Lawson2b: U = e^{tau A}(u + tau g(u)); u+ = e^{tau A}(u + tau/2 g(u)) + tau/2 g(U)."""
    g0 = be.g(u)
    U = be.expv(1.0, u + tau * g0)
    return be.expv(1.0, u + 0.5 * tau * g0) + 0.5 * tau * be.g(U)


def step_sl2(u, be, tau, alpha=ALPHA_SL2):
    """stabilized Lawson2: U = u + alpha tau e^{alpha tau A} F(u);
    u+ = u + tau e^{tau/2 A} F(u) + tau/(2 alpha) e^{tau A}(g(U) - g(u))."""
    F0 = be.F(u)
    g0 = be.g(u)
    U = u + alpha * tau * be.expv(alpha, F0)
    return u + tau * be.expv(0.5, F0) + tau / (2.0 * alpha) * be.expv(1.0, be.g(U) - g0)


def step_ee(u, be, tau):
    """exponential Euler: u+ = u + tau phi1(tau A) F(u)."""
    return u + tau * be.phi1v(be.F(u))


def step_erk2p2(u, be, tau):
    """ERK2 with phi2, c2 = 1: U = u + tau phi1 F(u); u+ = U + tau phi2 (g(U) - g(u))."""
    U = u + tau * be.phi1v(be.F(u))
    return U + tau * be.phi2v(be.g(U) - be.g(u))


def step_erk2p1(u, be, tau):
    """ERK2 with phi1, c2 = 1 (Appendix form): U = u + tau phi1 F(u);
    u+ = U + tau/2 phi1 (g(U) - g(u))."""
    U = u + tau * be.phi1v(be.F(u))
    return U + 0.5 * tau * be.phi1v(be.g(U) - be.g(u))


def step_etd2rk(u, be, tau):
    """ETD2RK (module docstring): U = e^{tau A} u + tau phi1 g(u); u+ = U + tau/2 phi1 (g(U) - g(u))."""
    g0 = be.g(u)
    U = be.expv(1.0, u) + tau * be.phi1v(g0)
    return U + 0.5 * tau * be.phi1v(be.g(U) - g0)


STEPS: Dict[str, Callable] = {
    "le": step_le, "sle": step_sle, "l2a": step_l2a, "l2b": step_l2b, "sl2": step_sl2,
    "ee": step_ee, "erk2p2": step_erk2p2, "erk2p1": step_erk2p1, "etd2rk": step_etd2rk,
    # the Appendix form of erk2p1, used with quadrature phi1 ("F-form")
    "erk2p1f": step_erk2p1,
}


def integrate(u0: np.ndarray, be, tau: float, steps: int, scheme: str) -> np.ndarray:
    step = STEPS[scheme]
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(steps):
        u = step(u, be, tau)
    return u


def rel_inf_error(u: np.ndarray, ref: np.ndarray) -> float:
    """relative infinity-norm error (Sec. 4.1)."""
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


class GridBackend:
    """Finite-difference backend of the schemes on one ADR problem (synth.Problem).

    phi="quad" uses the q-point Gauss-Legendre phi1; phi="exact" the joint eigenbasis,
    which is also what a problem with q = 0 (no quadrature nodes) asks for.
    """

    def __init__(self, prob, phi: str = "quad"):
        from .adr import extracted_amax, full_rhs, remainder
        from .expo import KronOperator
        self.prob = prob
        self.a_max = extracted_amax(prob.a)
        self.op = KronOperator(prob.n, self.a_max, prob.lam, prob.beta_bar, prob.tau)
        self._remainder, self._full = remainder, full_rhs
        self.phi = "exact" if prob.q == 0 else phi

    def expv(self, c, v):
        return self.op.expv(c, v)

    def g(self, v):
        p = self.prob
        return self._remainder(v, p.a, p.beta, p.r, p.lam, p.beta_bar, self.a_max)

    def F(self, v):
        p = self.prob
        return self._full(v, p.a, p.beta, p.r)

    def phi1v(self, v):
        if self.phi == "exact":
            return self.op.phi1v_exact(v)
        return self.op.phi1v_quad(v, self.prob.q)

    def phi2v(self, v):
        return self.op.phi2v_exact(v)


def solve(prob, steps=None, phi: str = "quad", scheme=None) -> np.ndarray:
    """Run the problem's scheme for ``steps`` (default prob.steps) steps from u0."""
    be = GridBackend(prob, phi=phi)
    return integrate(prob.u0, be, prob.tau, prob.steps if steps is None else steps,
                     scheme or prob.scheme)
