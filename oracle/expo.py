"""Matrix exponentials of Kronecker sums by mu-mode products, and phi1
(oracle; test infrastructure only).

Sec. 1 and Sec. 5.2: for a Kronecker sum A_d (+) ... (+) A_1,

    exp(A_d (+) ... (+) A_1) vec(V) = vec(V x_1 exp(A_1) x_2 ... x_d exp(A_d)),

where (V x_mu M)[.., j, ..] = sum_i M[j, i] V[.., i, ..] contracts the mu-th index.

1D factors: the paper does not say how exp(tau A_mu) is formed. Here the
closed form through the sine transform is used: a constant tridiagonal
Toeplitz matrix T (sub s, diagonal delta, super t, s*t > 0) is similar, via
D = diag(rho^j), rho = sqrt(s/t), to the symmetric tridiagonal matrix with
off-diagonal sigma = sign(t) sqrt(s t), whose eigenvectors are the columns of the
orthogonal DST-I matrix S[j,k] = sqrt(2/(n+1)) sin(j k pi/(n+1)) with eigenvalues
delta + 2 sigma cos(k pi/(n+1)). Hence exp(c T) = D S diag(exp(c ev)) S D^{-1}.
Two rewritings that are exact in real arithmetic keep the rounding at the level of
the data: the eigenvalues are evaluated as (delta + 2 sigma) - 4 sigma
sin^2(k pi/(2(n+1))) (half-angle identity), with delta + 2 sigma =
(delta^2 - 4 sigma^2)/(delta - 2 sigma) = 4 adv^2/(delta - 2 sigma) for
s = diff - adv, t = diff + adv, delta = -2 diff -- the cosine form loses about
2 |delta| u to cancellation in the smallest eigenvalues, which the stiffest
exponentials turn into relative errors near 1e-13; and the sine arguments
j k pi/(n+1) are reduced exactly, j k mod 2(n+1), before the multiplication by
pi/(n+1).

phi-functions (Sec. 1): phi1(z) = (e^z - 1)/z, phi2(z) = (phi1(z) - 1)/z.
phi1 of a Kronecker sum is not a product of 1D functions; it is evaluated
either exactly, pointwise in the joint eigenbasis, or by q-point Gauss-Legendre
quadrature of phi1(tau K) = int_0^1 exp(theta tau K) d theta (the quadrature is
not in the paper; its nodes are the Legendre roots mapped to [0,1]).

Pins: test_oracle_expo (factors vs scipy expm; mu-mode action vs brute-force
expm of the assembled Kronecker sum, nonsymmetric factors, non-cubic grids;
exact phi1 vs the augmented-matrix identity; quadrature exactness on
polynomials; closed-form sine-series evolution).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .adr import axis_of


def dst1_matrix(n: int) -> np.ndarray:
    """Orthogonal symmetric DST-I matrix S[j,k] = sqrt(2/(n+1)) sin(j k pi/(n+1)), j,k=1..n."""
    j = np.arange(1, n + 1)
    m = np.outer(j, j) % (2 * (n + 1))          # sin(x pi/(n+1)) has period 2(n+1) in x
    return np.sqrt(2.0 / (n + 1)) * np.sin(m * np.pi / (n + 1))


def toeplitz_eigen(n: int, a_max: float, lam: float, beta_bar: float):
    """Eigen-decomposition data of the 1D operator lam*a_max*D2 + beta_bar*D1 (centred FD).

    Returns (ev, left, right) with A_mu = left @ diag(ev) @ right.
    """
    h = 1.0 / (n + 1)
    diff = lam * a_max / h ** 2
    adv = beta_bar / (2.0 * h)
    s, delta, t = diff - adv, -2.0 * diff, diff + adv
    if s * t <= 0.0:
        raise NotImplementedError("closed form needs s*t > 0 (cell Peclet number below 2)")
    rho = np.sqrt(s / t)
    sigma = np.sign(t) * np.sqrt(s * t)
    k = np.arange(1, n + 1)
    # delta + 2 sigma cos(theta_k) without cancellation (module docstring)
    c0 = 4.0 * adv ** 2 / (delta - 2.0 * sigma) if delta != 2.0 * sigma else delta + 2.0 * sigma
    ev = c0 - 4.0 * sigma * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    S = dst1_matrix(n)
    jj = np.arange(1, n + 1).astype(np.float64)
    Dg = rho ** jj
    left = Dg[:, None] * S          # D S
    right = S / Dg[None, :]         # S D^{-1}
    return ev, left, right


def exp_factor(n: int, a_max: float, lam: float, beta_bar: float, ctau: float) -> np.ndarray:
    """exp(ctau * A_mu) for the 1D extracted operator, by the closed form above."""
    ev, left, right = toeplitz_eigen(n, a_max, lam, beta_bar)
    return (left * np.exp(ctau * ev)[None, :]) @ right


def mode_product(V: np.ndarray, M: np.ndarray, mu: int) -> np.ndarray:
    """V x_mu M: contract spatial index mu (x1 = 0) of V with the columns of M."""
    ax = axis_of(mu, V.ndim)
    return np.ascontiguousarray(np.moveaxis(np.tensordot(M, V, axes=([1], [ax])), 0, ax))


def tucker(V: np.ndarray, mats: Sequence[np.ndarray]) -> np.ndarray:
    """V x_1 M_1 x_2 M_2 (x_3 M_3), modes applied in order 1, 2, 3."""
    W = V
    for mu, M in enumerate(mats):
        W = mode_product(W, M, mu)
    return W


def phi1(z):
    """phi1(z) = (e^z - 1)/z with phi1(0) = 1 (expm1 keeps small |z| accurate)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def phi2(z):
    """phi2(z) = (phi1(z) - 1)/z = (e^z - 1 - z)/z^2; Taylor series for |z| < 0.5."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 0.5
    zs = z[small]
    acc = np.zeros_like(zs)
    fact = 2.0
    term = np.ones_like(zs)
    for k in range(0, 25):
        acc += term / fact
        term = term * zs
        fact *= (k + 3)
    out[small] = acc
    zl = z[~small]
    out[~small] = (np.expm1(zl) - zl) / zl ** 2
    return out


def gauss_legendre_01(q: int) -> Tuple[np.ndarray, np.ndarray]:
    """q-point Gauss-Legendre nodes theta_j and weights w_j on [0, 1]."""
    xi, om = np.polynomial.legendre.leggauss(q)
    return 0.5 * (xi + 1.0), 0.5 * om


class KronOperator:
    """The extracted operator A = A_d (+) ... (+) A_1 on one grid, with
    closed-form 1D exponentials and the joint eigenbasis."""

    def __init__(self, n: Sequence[int], a_max: float, lam: float, beta_bar: Sequence[float], tau: float):
        self.n = tuple(n)
        self.d = len(self.n)
        self.a_max, self.lam, self.tau = a_max, lam, tau
        self.beta_bar = tuple(beta_bar)
        self.eig = [toeplitz_eigen(self.n[mu], a_max, lam, self.beta_bar[mu]) for mu in range(self.d)]
        self._cache = {}

    def factors(self, c: float) -> List[np.ndarray]:
        """[exp(c tau A_1), ..., exp(c tau A_d)]"""
        key = float(c)
        if key not in self._cache:
            mats = []
            for mu in range(self.d):
                ev, left, right = self.eig[mu]
                mats.append((left * np.exp(c * self.tau * ev)[None, :]) @ right)
            self._cache[key] = mats
        return self._cache[key]

    def expv(self, c: float, V: np.ndarray) -> np.ndarray:
        """exp(c tau A) V by mu-mode products."""
        return tucker(V, self.factors(c))

    def _joint_eigenvalues(self) -> np.ndarray:
        """sum_mu ev_mu[k_mu] on the C-ordered index grid (k_d .. k_1)."""
        d = self.d
        total = np.zeros(tuple(reversed(self.n)))
        for mu in range(d):
            shape = [1] * d
            shape[axis_of(mu, d)] = self.n[mu]
            total = total + self.eig[mu][0].reshape(shape)
        return total

    def funv(self, f, V: np.ndarray) -> np.ndarray:
        """f(tau A) V through the joint eigenbasis: transform, scale pointwise, transform back."""
        Vh = tucker(V, [self.eig[mu][2] for mu in range(self.d)])
        Vh = Vh * f(self.tau * self._joint_eigenvalues())
        return tucker(Vh, [self.eig[mu][1] for mu in range(self.d)])

    def phi1v_exact(self, V: np.ndarray) -> np.ndarray:
        return self.funv(phi1, V)

    def phi2v_exact(self, V: np.ndarray) -> np.ndarray:
        return self.funv(phi2, V)

    def phi1v_quad(self, V: np.ndarray, q: int) -> np.ndarray:
        """sum_j w_j exp(theta_j tau A) V, the q-point Gauss-Legendre rule for phi1."""
        th, w = gauss_legendre_01(q)
        out = np.zeros_like(V)
        for tj, wj in zip(th, w):
            out += wj * self.expv(tj, V)
        return out
