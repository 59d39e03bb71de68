"""The three-dimensional problem of Sec. 5.2 and the boundary and diffusion forms it
needs (oracle; test infrastructure only: tests and the benchmark's CPU baseline use
it, the product path never does).

Equation (eq:adr3d): u_t = a(x) Lap u + b sum_mu d_mu u + r(u) on (0,1)^3, homogeneous
Dirichlet data on the faces x_mu = 0 and homogeneous Neumann data on the faces
x_mu = 1, a(x) = exp(-|x - 1/2|^2)/10, r(u) = u(1 + u^2), u0 = (27/4)^3 prod x(1-x)^2.
Equation (eq:adr3dstab) splits it as A = lam a_max Lap + b sum d_mu (advection wholly
in A) and g = (a - lam a_max) Lap u + r(u).

Discretization (a reading of "standard second order centered finite differences"
with N points per direction, confirmed by reproducing every printed point of
Figure fig:adr3d_diffl, see tests/test_oracle_adr3d.py):
  * an axis with Neumann data at x = 1 has the N unknowns x_i = i h, h = 1/N,
    i = 1..N (the Neumann face carries an unknown); an axis with Dirichlet data at
    both ends keeps n unknowns at x_i = i/(n+1);
  * centred differences everywhere; the value beyond the Neumann face is the
    mirror ghost u_{N+1} = u_{N-1} (for N = 1 the mirror is the Dirichlet value 0),
    zero ghosts on Dirichlet faces;
  * diffusion in non-divergence form a Lap u (the problem's own), or in the flux
    form div(a grad u) with face means of the nodal a (the other workloads), using
    the given nodal values of a on the padded node set (for a Neumann axis the
    padded node N+1 holds the mirror value a(x_{N-1}), written by the problem
    generator).
The 1D matrices A_mu follow from the same ghost rule (the Neumann row reads
[..., 2, -2]/h^2, its centred advection cancels), and their exponentials are taken
with scipy.linalg.expm on the dense matrices. All-Dirichlet flux-form problems reduce
to oracle.adr, which is written separately: the two agree (a pin).

Exact phi functions (problems with q = 0) go through numpy's dense eigen-decomposition of
every A_mu.

Pins: tests/test_oracle_adr3d.py (the printed errors of Figure fig:adr3d_diffl for
LE, SLE, L2a and SL2 at both advection speeds; the closed-form eigenpairs of the
Dirichlet-Neumann second difference; agreement with oracle.adr on all-Dirichlet
flux-form problems; F = A u + g; phi1 and phi2 of the Kronecker sum against the
augmented-matrix exponential identities on small mixed grids).
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import scipy.linalg

DIRICHLET, NEUMANN = 0, 1     # per-axis data at x = 1 (x = 0 is always Dirichlet)


def spacing(n: int, bc: int) -> float:
    """Mesh width of an axis with n unknowns."""
    return 1.0 / n if bc == NEUMANN else 1.0 / (n + 1)


def nodes(n: int, bc: int) -> np.ndarray:
    """Coordinates of the n unknowns of an axis."""
    return spacing(n, bc) * np.arange(1, n + 1)


def _axis(mu: int, d: int) -> int:
    return d - 1 - mu


def ghost_pad(u: np.ndarray, bcs: Sequence[int]) -> np.ndarray:
    """u with one ghost layer on both sides of every spatial axis: zero on Dirichlet
    faces, the mirror value u[n-2] beyond a Neumann face."""
    d = u.ndim
    out = u
    for mu in range(d):
        ax = _axis(mu, d)
        n = u.shape[ax]
        lo = np.zeros_like(np.take(out, [0], axis=ax))
        hi = np.take(out, [n - 2], axis=ax) if (bcs[mu] == NEUMANN and n >= 2) else np.zeros_like(lo)
        out = np.concatenate([lo, out, hi], axis=ax)
    return out


def _nb(arr: np.ndarray, ax: int, off: int) -> np.ndarray:
    """The padded array's values at offset off along axis ax, aligned with the core."""
    sl = [slice(1, -1)] * arr.ndim
    sl[ax] = slice(1 + off, arr.shape[ax] - 1 + off)
    return arr[tuple(sl)]


def reaction(u: np.ndarray, r: Sequence[float]) -> np.ndarray:
    return r[0] + u * (r[1] + u * (r[2] + u * r[3]))


def remainder(u: np.ndarray, a: np.ndarray, beta: Sequence[float], r: Sequence[float], lam: float,
              beta_bar: Sequence[float], a_max: float, bcs: Sequence[int], form: str) -> np.ndarray:
    """g(u) = diffusion with coefficient (a - lam a_max) + (beta - beta_bar) . grad u + r(u)
    (eq. (eq:adr3dstab) for form = "nondiv"; eq. (eq:nonlin) for form = "flux")."""
    d = u.ndim
    up = ghost_pad(u, bcs)
    core = tuple(slice(1, -1) for _ in range(d))
    ac = a[core]
    la = lam * a_max
    g = reaction(u, r).astype(float)
    for mu in range(d):
        ax = _axis(mu, d)
        h = spacing(u.shape[ax], bcs[mu])
        upp, upm = _nb(up, ax, 1), _nb(up, ax, -1)
        if form == "nondiv":
            g = g + (ac - la) * (upp - 2.0 * u + upm) / h ** 2
        else:
            ap, am = _nb(a, ax, 1), _nb(a, ax, -1)
            g = g + ((0.5 * (ac + ap) - la) * (upp - u) - (0.5 * (ac + am) - la) * (u - upm)) / h ** 2
        g = g + (beta[mu] - beta_bar[mu]) * (upp - upm) / (2.0 * h)
    return g


def full_rhs(u: np.ndarray, a: np.ndarray, beta: Sequence[float], r: Sequence[float], bcs: Sequence[int],
             form: str) -> np.ndarray:
    """F(u): the whole right-hand side (nothing extracted)."""
    return remainder(u, a, beta, r, 0.0, [0.0] * u.ndim, 0.0, bcs, form)


def operator_1d(n: int, bc: int, lam_amax: float, beta_bar: float) -> np.ndarray:
    """Dense A_mu = lam a_max d2/dx2 + beta_bar d/dx by centred differences with the
    ghost rule of ghost_pad."""
    h = spacing(n, bc)
    dif, adv = lam_amax / h ** 2, beta_bar / (2.0 * h)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = -2.0 * dif
        if i > 0:
            A[i, i - 1] += dif - adv
        if i + 1 < n:
            A[i, i + 1] += dif + adv
        elif bc == NEUMANN and n >= 2:
            A[i, i - 1] += dif + adv          # the mirror ghost u_{n+1} = u_{n-1}
    return A


def tucker(V: np.ndarray, mats: Sequence[np.ndarray]) -> np.ndarray:
    """V x_1 M_1 x_2 M_2 (x_3 M_3): contract spatial index mu with the columns of M_mu."""
    W = V
    d = V.ndim
    for mu, M in enumerate(mats):
        W = np.moveaxis(np.tensordot(M, W, axes=([1], [_axis(mu, d)])), 0, _axis(mu, d))
    return W


class Backend:
    """Scheme backend (expv, g, F) for a problem with per-axis boundary data and a
    diffusion form (fields bc and form of synth.Problem)."""

    def __init__(self, prob):
        self.p = prob
        self.bcs = tuple(prob.bc)
        self.form = prob.form
        self.a_max = float(np.max(prob.a))
        self.A = [operator_1d(prob.n[mu], self.bcs[mu], prob.lam * self.a_max, prob.beta_bar[mu])
                  for mu in range(prob.d)]
        self._E = {}
        self._eigs = None
        self.phi = "exact" if prob.q == 0 else "quad"

    def factors(self, c: float):
        if c not in self._E:
            self._E[c] = [scipy.linalg.expm(c * self.p.tau * A) for A in self.A]
        return self._E[c]

    def expv(self, c, v):
        return tucker(v, self.factors(c))

    def g(self, v):
        p = self.p
        return remainder(v, p.a, p.beta, p.r, p.lam, p.beta_bar, self.a_max, self.bcs, self.form)

    def F(self, v):
        p = self.p
        return full_rhs(v, p.a, p.beta, p.r, self.bcs, self.form)

    def eigen(self):
        """A_mu = V_mu diag(lam_mu) V_mu^-1 for every axis, from numpy's general dense
        eigensolver (a different route from the closed forms the GPU path uses); the
        spectra are real for the problems here (|beta_bar| h < 2 lam a_max)."""
        if self._eigs is None:
            self._eigs = []
            for A in self.A:
                lam, V = np.linalg.eig(A)
                if np.max(np.abs(lam.imag)) > 1e-10 * max(1.0, float(np.max(np.abs(lam)))):
                    raise ValueError("complex spectrum: no real eigenbasis for exact phi functions")
                self._eigs.append((lam.real, V.real, np.linalg.inv(V.real)))
        return self._eigs

    def funv(self, f, v):
        """f(tau A) v for the Kronecker sum A = A_d + ... + A_1: transform with V_mu^-1 along
        every axis, scale by f(tau (lam_1 + ... + lam_d)), transform back with V_mu."""
        eigs = self.eigen()
        d = v.ndim
        W = tucker(v, [e[2] for e in eigs])
        total = np.zeros(W.shape)
        for mu in range(d):
            shape = [1] * d
            shape[_axis(mu, d)] = eigs[mu][0].size
            total = total + eigs[mu][0].reshape(shape)
        return tucker(W * f(self.p.tau * total), [e[1] for e in eigs])

    def phi1v(self, v):
        """phi1(tau A) v: exact (funv) for a problem without quadrature nodes (q = 0), else
        the q-point Gauss-Legendre rule sum_j w_j exp(theta_j tau A) v."""
        if self.phi == "exact":
            from .expo import phi1
            return self.funv(phi1, v)
        from .expo import gauss_legendre_01
        th, w = gauss_legendre_01(self.p.q)
        out = np.zeros_like(v)
        for tj, wj in zip(th, w):
            out += wj * self.expv(tj, v)
        return out

    def phi2v(self, v):
        from .expo import phi2
        return self.funv(phi2, v)


def solve(prob, steps=None, scheme=None) -> np.ndarray:
    """prob.scheme from prob.u0: Lawson schemes; ETD2RK / ERK2P1 with quadrature phi1
    (q > 0) or exact phi1 (q = 0); EE and erk2p2 (exact phi functions, q = 0)."""
    from .schemes import integrate
    sch = scheme or prob.scheme
    if sch in ("ee", "erk2p2", "erk2p1") and prob.q != 0:
        raise ValueError(f"{sch} needs exact phi functions (q = 0)")
    return integrate(prob.u0, Backend(prob), prob.tau, prob.steps if steps is None else steps, sch)
