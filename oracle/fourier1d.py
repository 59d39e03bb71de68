"""Periodic 1D pseudo-spectral setting of Sec. 4.1 (oracle; test infrastructure only).

Equation (eq:adlinearzero): u_t = a(x) u_xx on (-pi, pi), periodic,
a(x) = 1 + 10 sin^2 x, u0 = sin x, rewritten as (eq:ex0stab) with
A = lam a_max d^2/dx^2 and g(u) = (a - lam a_max) u_xx, a_max = 11. Derivatives
and matrix functions of A are pointwise on the Fourier coefficients.

This backend exists only to run the step code of ``schemes`` on the paper's own
worked example and compare with its printed errors; it is not part of the
mu-mode path.

Exact reference: the solution is odd and a(x) = 6 - 5 cos 2x couples sin(kx)
only to sin((k +- 2)x):
    a (sin kx)'' = -6 k^2 sin kx + 2.5 k^2 [sin((k+2)x) + sin((k-2)x)],
with sin(-x) = -sin x for k = 1. The semi-discrete solution (N = 2^12 modes, no
aliasing at the retained wavenumbers) is therefore exp(T M) e_1 in the basis
sin(x), sin(3x), ..., which scipy's expm evaluates on a small matrix.
"""
from __future__ import annotations

import numpy as np

from .expo import phi1, phi2


class Fourier1D:
    def __init__(self, N: int, lam: float, tau: float):
        self.N = N
        self.x = -np.pi + 2.0 * np.pi * np.arange(N) / N
        self.a = 1.0 + 10.0 * np.sin(self.x) ** 2
        self.a_max = 11.0
        self.lam, self.tau = lam, tau
        self.k2 = np.arange(N // 2 + 1, dtype=np.float64) ** 2     # rfft wavenumbers squared
        self.symbol = -self.lam * self.a_max * self.k2              # eigenvalues of A

    def uxx(self, v):
        return np.fft.irfft(-self.k2 * np.fft.rfft(v), n=self.N)

    def g(self, v):
        return (self.a - self.lam * self.a_max) * self.uxx(v)

    def F(self, v):
        return self.a * self.uxx(v)

    def _mult(self, mult, v):
        return np.fft.irfft(mult * np.fft.rfft(v), n=self.N)

    def expv(self, c, v):
        return self._mult(np.exp(c * self.tau * self.symbol), v)

    def phi1v(self, v):
        return self._mult(phi1(self.tau * self.symbol), v)

    def phi2v(self, v):
        return self._mult(phi2(self.tau * self.symbol), v)


def exact_solution(x: np.ndarray, T: float, kmax: int = 401) -> np.ndarray:
    """u(T, x) for u0 = sin x by expm of the odd-sine Galerkin matrix (modes 1, 3, .., kmax)."""
    from scipy.linalg import expm
    ks = np.arange(1, kmax + 1, 2)
    m = len(ks)
    M = np.zeros((m, m))
    for j, k in enumerate(ks):
        M[j, j] += -6.0 * k ** 2
        if j + 1 < m:
            M[j + 1, j] += 2.5 * k ** 2          # sin((k+2)x)
        if k >= 3:
            M[j - 1, j] += 2.5 * k ** 2          # sin((k-2)x)
        else:
            M[j, j] += -2.5 * k ** 2             # sin(-x) = -sin x
    b0 = np.zeros(m)
    b0[0] = 1.0
    b = expm(T * M) @ b0
    return np.sin(np.outer(x, ks)) @ b
