"""Periodic pseudo-spectral problems of Sec. 4.1, 4.2 and 5.1 (oracle; test
infrastructure only: tests and the benchmark's CPU baseline use it, the product path
never does).

Equation (eq:adr) on a periodic box with a diagonal diffusion tensor
diag(a_11(x), .., a_dd(x)) and a velocity field b(x):

    u_t = sum_mu d_mu(a_mumu d_mu u) + div(b u) + r(u)     ("flux" form), or
    u_t = sum_mu a_mumu d_mumu u + div(b u) + r(u)          ("nondiv" form, eq. (eq:adlinearzero)).

Splitting (eq. (eq:fullstab)): A = sum_mu (lam a_mumu^max d_mumu + beta_mu d_mu) with
a^max the maximum of each a_mumu over the grid and beta the extracted velocity (given
by the caller: for eq. (eq:amaxbeta) the mean of b_mu + d_mu a_mumu), and
g = F - A u written out as
    sum_mu d_mu((a_mumu - lam a^max_mumu) d_mu u) + sum_mu d_mu((b_mu - beta_mu) u) + r(u)
(flux form; nondiv: (a_mumu - lam a^max_mumu) d_mumu u). F(u) = A u + g(u) exactly.

Discretization (the paper's Fourier pseudo-spectral setting): n_mu equispaced points
per period L_mu, x_j = x0 + j L_mu / n_mu; derivatives are products with the Fourier
symbols of the discrete Fourier transform along the axis, i kappa for d_mu and
-kappa^2 for d_mumu, kappa = 2 pi m / L_mu for the integer wavenumbers m of the
transform. For even n the first-derivative symbol is zero at the Nyquist wavenumber
m = n/2 (the derivative of a real grid function stays real) and the second-derivative
symbol is -(pi n / L)^2 there. Everything in this module goes through numpy's FFT; the
exponential of A is the pointwise exponential of its symbol.

A problem with no velocity field uses the constant velocity beta of the problem instead
(then div(b u) = beta . grad u).

Pins: tests/test_oracle_spectral.py (the printed errors of Figure fig:ad1dex0_diffdeltaa
through this backend; derivatives and exponentials of trigonometric polynomials in
closed form; F = A u + g; the lambda values of Table tab:adr2d_lambdaopt and the printed
errors of Figure fig:adr2d_diffl for the problem of Sec. 5.1).
"""
from __future__ import annotations

import numpy as np


def wavenumbers(n: int, length: float):
    """(first-derivative symbol factor kappa1, second-derivative kappa^2) per transform
    index for n points on a period of the given length."""
    m = np.fft.fftfreq(n, 1.0 / n)            # 0, 1, .., n/2 - 1, -n/2, .., -1 (even n)
    s = 2.0 * np.pi / length
    k1 = s * m
    if n % 2 == 0:
        k1[n // 2] = 0.0
    k2 = (s * m) ** 2
    return k1, k2


def phi_complex(k: int, z) -> np.ndarray:
    """phi_k(z) = sum_j z^j / (j + k)! (k = 1, 2) for complex z: the series for |z| < 1/2,
    (e^z - 1)/z and (e^z - 1 - z)/z^2 otherwise."""
    z = np.asarray(z, dtype=complex)
    out = np.empty_like(z)
    small = np.abs(z) < 0.5
    zs = z[small]
    acc = np.zeros_like(zs)
    term = np.ones_like(zs)
    fact = float(np.prod(np.arange(1, k + 1)))
    for j in range(25):
        acc += term / fact
        term = term * zs
        fact *= j + k + 1
    out[small] = acc
    zl = z[~small]
    out[~small] = (np.exp(zl) - 1.0) / zl if k == 1 else (np.exp(zl) - 1.0 - zl) / zl ** 2
    return out


def grid(n: int, length: float, x0: float = 0.0) -> np.ndarray:
    return x0 + length / n * np.arange(n)


class Spectral:
    """Scheme backend (expv, g, F, phi1v, phi2v) for a periodic problem (synth.Problem
    with every bc periodic: ``a`` of shape (d, *grid), ``velocity`` None or of the same
    shape, ``length`` the periods)."""

    def __init__(self, prob, phi: str = "quad"):
        self.p = prob
        d = prob.d
        self.d = d
        self.shape = prob.u0.shape
        self.phi = phi
        a = np.asarray(prob.a, dtype=float)
        self.a = [a[mu] for mu in range(d)]
        self.vel = None if prob.velocity is None else [np.asarray(prob.velocity[mu], dtype=float) for mu in range(d)]
        self.a_max = [float(np.max(self.a[mu])) for mu in range(d)]
        self.k1, self.k2, self.sym = [], [], []
        for mu in range(d):
            k1, k2 = wavenumbers(prob.n[mu], prob.length[mu])
            self.k1.append(k1)
            self.k2.append(k2)
            self.sym.append(prob.lam * self.a_max[mu] * (-k2) + 1j * prob.beta_bar[mu] * k1)
        # symbol of A on the full transform grid (array axis d-1-mu is x_mu)
        S = np.zeros(self.shape, dtype=complex)
        for mu in range(d):
            S = S + self._along(self.sym[mu], mu)
        self.S = S

    def _along(self, vec, mu):
        sh = [1] * self.d
        sh[self.d - 1 - mu] = -1
        return np.reshape(vec, sh)

    def _mult(self, v, mu, mult):
        ax = self.d - 1 - mu
        return np.real(np.fft.ifft(self._along(mult, mu) * np.fft.fft(v, axis=ax), axis=ax))

    def d1(self, v, mu):
        return self._mult(v, mu, 1j * self.k1[mu])

    def d2(self, v, mu):
        return self._mult(v, mu, -self.k2[mu])

    def A(self, v):
        return np.real(np.fft.ifftn(self.S * np.fft.fftn(v)))

    def g(self, v):
        p = self.p
        out = p.r[0] + v * (p.r[1] + v * (p.r[2] + v * p.r[3]))
        for mu in range(self.d):
            c = self.a[mu] - p.lam * self.a_max[mu]
            if p.form == "nondiv":
                out = out + c * self.d2(v, mu)
            else:
                out = out + self.d1(c * self.d1(v, mu), mu)
            if self.vel is not None:
                out = out + self.d1((self.vel[mu] - p.beta_bar[mu]) * v, mu)
            else:
                out = out + (p.beta[mu] - p.beta_bar[mu]) * self.d1(v, mu)
        return out

    def F(self, v):
        return self.A(v) + self.g(v)

    def expv(self, c, v):
        return np.real(np.fft.ifftn(np.exp(c * self.p.tau * self.S) * np.fft.fftn(v)))

    def _phi_exact(self, k, v):
        f = phi_complex(k, self.p.tau * self.S)
        return np.real(np.fft.ifftn(f * np.fft.fftn(v)))

    def phi1v(self, v):
        """phi1(tau A) v: exact (pointwise on the symbol) or the q-point Gauss-Legendre
        quadrature sum_j w_j exp(theta_j tau A) v of the product path."""
        if self.phi == "exact":
            return self._phi_exact(1, v)
        from .expo import gauss_legendre_01
        th, w = gauss_legendre_01(self.p.q)
        out = np.zeros_like(v)
        for tj, wj in zip(th, w):
            out += wj * self.expv(tj, v)
        return out

    def phi2v(self, v):
        return self._phi_exact(2, v)


def solve(prob, steps=None, scheme=None, phi: str = "quad") -> np.ndarray:
    """prob.scheme from prob.u0 on the periodic problem."""
    from .schemes import integrate
    sch = scheme or prob.scheme
    return integrate(prob.u0, Spectral(prob, phi=phi), prob.tau, prob.steps if steps is None else steps, sch)
