"""Extraction of the constant-coefficient operator and the finite-difference
remainder (oracle; test infrastructure only).

Sec. 3, equations (eq:adr_equiv), (eq:linop), (eq:nonlin), (eq:amaxbeta): the
semilinear ADR equation u_t = div(a grad u) + div(b u) + r(u) is rewritten as
u_t = A u + g(u) with

    A u = lam * a_max * Laplacian(u) + beta_bar . grad u
    g(u) = div((a - lam*a_max) grad u) + div((b - beta_bar) u) + r(u).

Sec. 5.2: on a tensor grid, second-order centred finite differences turn A into
a Kronecker sum A_d (+) ... (+) A_1 of 1D matrices, one per axis.

Discrete readings (the paper does not spell the stencil out):
  * conservative flux form, face coefficient = arithmetic mean of the two
    nodal values of a; homogeneous Dirichlet data as zero ghost values;
  * constant velocity b = beta, so div(beta u) = beta . grad u, centred;
  * a_max is the maximum over every sampled node, boundary nodes included.

Pins: test_oracle_stencil (quadratic fields are differentiated exactly, the
constant-a reduction g = (a - lam a_max) Lap_h u, second-order consistency for
manufactured fields, F = A_h u + g).
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def mesh_widths(n: Sequence[int]) -> Tuple[float, ...]:
    """h_mu = 1/(n_mu + 1) for interior sizes listed x1 first."""
    return tuple(1.0 / (m + 1) for m in n)


def axis_of(mu: int, d: int) -> int:
    """numpy axis of spatial direction mu (0-based, x1 = 0) in a C-ordered array."""
    return d - 1 - mu


def extracted_amax(a: np.ndarray) -> float:
    """a_max of equation (eq:amaxbeta): max of a over all sampled nodes."""
    return float(np.max(a))


def operator_1d(n: int, a_max: float, lam: float, beta_bar: float) -> np.ndarray:
    """Dense 1D matrix A_mu: centred FD of lam*a_max*d2/dx2 + beta_bar*d/dx with
    homogeneous Dirichlet data on n interior points (Sec. 5.2)."""
    h = 1.0 / (n + 1)
    diff = lam * a_max / h ** 2
    adv = beta_bar / (2.0 * h)
    K = np.zeros((n, n))
    for i in range(n):
        K[i, i] = -2.0 * diff
        if i > 0:
            K[i, i - 1] = diff - adv
        if i + 1 < n:
            K[i, i + 1] = diff + adv
    return K


def _shift(arr: np.ndarray, ax: int, off: int) -> Tuple[slice, ...]:
    """index of the interior block shifted by ``off`` along ``ax`` in a padded array."""
    idx = [slice(1, -1)] * arr.ndim
    s = 1 + off
    e = arr.shape[ax] - 1 + off
    idx[ax] = slice(s, e)
    return tuple(idx)


def _pad_dirichlet(u: np.ndarray) -> np.ndarray:
    return np.pad(u, 1, mode="constant", constant_values=0.0)


def reaction(u: np.ndarray, r: Sequence[float]) -> np.ndarray:
    """r(u) = r0 + r1 u + r2 u^2 + r3 u^3."""
    return r[0] + r[1] * u + r[2] * u ** 2 + r[3] * u ** 3


def remainder(u: np.ndarray, a: np.ndarray, beta: Sequence[float], r: Sequence[float],
              lam: float, beta_bar: Sequence[float], a_max: float) -> np.ndarray:
    """g(u) of equation (eq:nonlin), discretised as a flux-form 2d+1-point stencil.

    Diffusion part per axis: [(abar+ - lam a_max)(u+ - u) - (abar- - lam a_max)(u - u-)]/h^2,
    advection part: (beta - beta_bar)(u+ - u-)/(2h), plus the pointwise reaction.
    """
    d = u.ndim
    n = tuple(reversed(u.shape))
    hs = mesh_widths(n)
    U = _pad_dirichlet(u)
    c = tuple([slice(1, -1)] * d)
    out = reaction(u, r).astype(np.float64)
    for mu in range(d):
        ax = axis_of(mu, d)
        h = hs[mu]
        p = _shift(U, ax, +1)
        m = _shift(U, ax, -1)
        a_p = 0.5 * (a[c] + a[p]) - lam * a_max
        a_m = 0.5 * (a[c] + a[m]) - lam * a_max
        out += (a_p * (U[p] - U[c]) - a_m * (U[c] - U[m])) / h ** 2
        out += (beta[mu] - beta_bar[mu]) * (U[p] - U[m]) / (2.0 * h)
    return out


def full_rhs(u: np.ndarray, a: np.ndarray, beta: Sequence[float], r: Sequence[float]) -> np.ndarray:
    """F(u): the unsplit discrete right-hand side div(a grad u) + beta.grad u + r(u)
    (Appendix, abstract form u' = F(u)), written out on its own, not as A u + g."""
    d = u.ndim
    n = tuple(reversed(u.shape))
    hs = mesh_widths(n)
    U = _pad_dirichlet(u)
    c = tuple([slice(1, -1)] * d)
    out = reaction(u, r).astype(np.float64)
    for mu in range(d):
        ax = axis_of(mu, d)
        h = hs[mu]
        p = _shift(U, ax, +1)
        m = _shift(U, ax, -1)
        a_p = 0.5 * (a[c] + a[p])
        a_m = 0.5 * (a[c] + a[m])
        out += (a_p * (U[p] - U[c]) - a_m * (U[c] - U[m])) / h ** 2
        out += beta[mu] * (U[p] - U[m]) / (2.0 * h)
    return out


def apply_kron_sum(u: np.ndarray, mats: Sequence[np.ndarray]) -> np.ndarray:
    """(A_d (+) ... (+) A_1) vec(u) as a sum of mode products (no exponential)."""
    d = u.ndim
    out = np.zeros_like(u)
    for mu, M in enumerate(mats):
        ax = axis_of(mu, d)
        out += np.moveaxis(np.tensordot(M, u, axes=([1], [ax])), 0, ax)
    return out
