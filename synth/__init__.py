"""Seeded synthetic inputs for the advection-diffusion-reaction workloads.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
problem data only -- coefficient fields sampled on the grid, initial data,
constant parameters, request streams -- and none of the time-stepping or
matrix-function arithmetic of the method.

Problem class (Sec. 3, equation (eq:adr), restricted to the workloads here):

    u_t = div(a(x) grad u) + beta . grad u + r(u)   on (0,1)^d,  u = 0 on the boundary,

with a scalar diffusion coefficient a(x) > 0, a constant velocity beta, and a
cubic reaction r(u) = r0 + r1 u + r2 u^2 + r3 u^3 (covers u(1-u) and u^2(1-u)).

Grid conventions (shared by both sides):
  * n_mu interior points along axis mu, mesh width h_mu = 1/(n_mu + 1),
    nodes x_{mu,i} = i*h_mu for i = 0..n_mu+1 (0 and n_mu+1 are boundary nodes);
  * arrays are C-ordered with x1 fastest: a 3D grid function has numpy shape
    (n3, n2, n1), a 2D one (n2, n1) -- the column-major vec() of the paper's
    tensor V (Sec. 5.2) is the same memory;
  * the diffusion coefficient is sampled on all nodes including the boundary,
    shape (n3+2, n2+2, n1+2).

Random fields are sine series s(x) = sum_k c_k prod_mu sin(k_mu pi x_mu) with
c_k ~ N(0,1)/|k|^2, drawn from numpy's PCG64 ``default_rng(seed)``. The draw
order is fixed: diffusion-field coefficients first, then initial-data
coefficients.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# reaction presets r(u) = r0 + r1 u + r2 u^2 + r3 u^3
R_LOGISTIC = (0.0, 1.0, -1.0, 0.0)      # u(1-u)
R_CUBIC = (0.0, 0.0, 1.0, -1.0)         # u^2(1-u)
R_NONE = (0.0, 0.0, 0.0, 0.0)


@dataclass
class Problem:
    """One semilinear ADR solve on (0,1)^d with homogeneous Dirichlet data.

    ``n`` lists interior sizes x1 first. ``a`` is nodal including boundary
    (C order, x1 fastest); ``u0`` is interior only. ``lam`` and ``beta_bar``
    are the extraction parameters of equation (eq:linop): the extracted
    operator is lam*max(a)*Laplacian + beta_bar . grad.
    """
    d: int
    n: Tuple[int, ...]
    a: np.ndarray
    u0: np.ndarray
    beta: Tuple[float, ...]
    r: Tuple[float, float, float, float]
    tau: float
    steps: int
    scheme: str = "l2b"          # "le", "l2b", "etd2rk", "erk2p1f"
    q: int = 4                   # Gauss-Legendre nodes for phi1
    lam: float = 1.0
    beta_bar: Tuple[float, ...] = ()
    name: str = ""
    # per axis: 0 = Dirichlet data at both ends, 1 = Dirichlet at x = 0 and homogeneous
    # Neumann at x = 1 (then the n unknowns sit at i/n, i = 1..n, and the padded node
    # n + 1 of ``a`` holds the mirror value a(x_{n-1}))
    bc: Tuple[int, ...] = ()
    # diffusion term: "flux" = div(a grad u), "nondiv" = a Lap u
    form: str = "flux"
    # periodic problems (every bc = 2): the period of each axis; ``a`` then holds the
    # diagonal diffusion tensor on the periodic grid, shape (d, *grid), and ``velocity``
    # (None or the same shape) a velocity field entering as div(velocity u)
    length: Tuple[float, ...] = ()
    velocity: Optional[np.ndarray] = None

    def __post_init__(self):
        if not self.beta_bar:
            self.beta_bar = tuple(0.0 for _ in range(self.d))
        if not self.bc:
            self.bc = tuple(0 for _ in range(self.d))

    @property
    def dof(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self) -> Tuple[int, ...]:
        """numpy shape of a grid function (slowest axis first)."""
        return tuple(reversed(self.n))

    @property
    def node_shape(self) -> Tuple[int, ...]:
        return tuple(m + 2 for m in reversed(self.n))


def _sine_basis(kmax: int, n: int, include_boundary: bool) -> np.ndarray:
    """rows k=1..kmax of sin(k pi x_i) on the nodes of an axis with n interior points."""
    h = 1.0 / (n + 1)
    idx = np.arange(0, n + 2) if include_boundary else np.arange(1, n + 1)
    x = idx * h
    k = np.arange(1, kmax + 1)[:, None]
    return np.sin(np.pi * k * x[None, :])


def sine_series(rng: np.random.Generator, n: Sequence[int], kmax: Sequence[int],
                include_boundary: bool) -> np.ndarray:
    """Seeded sine series with N(0,1)/|k|^2 coefficients, C order (x1 fastest).

    ``n`` and ``kmax`` list axes x1 first. The coefficient array is drawn in C
    order over (k_d, ..., k_1).
    """
    d = len(n)
    kshape = tuple(reversed(list(kmax)))                       # (k_d .. k_1)
    grids = np.meshgrid(*[np.arange(1, km + 1) for km in kshape], indexing="ij")
    ksq = sum(g.astype(np.float64) ** 2 for g in grids)
    c = rng.standard_normal(kshape) / ksq
    bases = [_sine_basis(kmax[mu], n[mu], include_boundary) for mu in range(d)]
    if d == 2:
        # s[i2, i1] = sum c[k2,k1] B2[k2,i2] B1[k1,i1]
        return np.einsum("ba,bj,ak->jk", c, bases[1], bases[0], optimize=True)
    if d == 3:
        return np.einsum("cba,ci,bj,ak->ijk", c, bases[2], bases[1], bases[0], optimize=True)
    raise ValueError("d must be 2 or 3")


def smooth_problem(n: Sequence[int], seed: int, *, a_amp: float = 0.9, a_kmax: int = 4,
                   u_kmax: int = 8, beta: Optional[Sequence[float]] = None,
                   r: Sequence[float] = R_CUBIC, tau: float = 1e-3, steps: int = 10,
                   scheme: str = "l2b", q: int = 4, lam: float = 1.0,
                   beta_bar: Optional[Sequence[float]] = None, name: str = "") -> Problem:
    """a = 1 + a_amp*tanh(s_a) (modes <= a_kmax), u0 = s_u/max|s_u| (modes <= u_kmax)."""
    n = tuple(int(m) for m in n)
    d = len(n)
    rng = np.random.default_rng(seed)
    s_a = sine_series(rng, n, [a_kmax] * d, include_boundary=True)
    s_u = sine_series(rng, n, [u_kmax] * d, include_boundary=False)
    a = 1.0 + a_amp * np.tanh(s_a)
    u0 = s_u / np.max(np.abs(s_u))
    if beta is None:
        beta = (10.0,) * d
    return Problem(d=d, n=n, a=np.ascontiguousarray(a), u0=np.ascontiguousarray(u0),
                   beta=tuple(float(b) for b in beta), r=tuple(float(x) for x in r),
                   tau=float(tau), steps=int(steps), scheme=scheme, q=int(q), lam=float(lam),
                   beta_bar=tuple(beta_bar) if beta_bar is not None else (), name=name)


def anisotropic_problem(n: int, seed: int, *, tau: float, steps: int, scheme: str = "etd2rk",
                        q: int = 6, name: str = "") -> Problem:
    """a = 0.01 + 0.995*(1 + tanh(3 s)) in (0.01, 2), s with modes k1<=8, k2,k3<=2."""
    nn = (n, n, n)
    rng = np.random.default_rng(seed)
    s_a = sine_series(rng, nn, [8, 2, 2], include_boundary=True)
    s_u = sine_series(rng, nn, [8, 8, 8], include_boundary=False)
    a = 0.01 + 0.995 * (1.0 + np.tanh(3.0 * s_a))
    u0 = s_u / np.max(np.abs(s_u))
    return Problem(d=3, n=nn, a=np.ascontiguousarray(a), u0=np.ascontiguousarray(u0),
                   beta=(10.0, 10.0, 10.0), r=R_CUBIC, tau=tau, steps=steps, scheme=scheme,
                   q=q, name=name)


def constant_problem(n: Sequence[int], seed: int, *, a_const: float, u_kmax: int = 3,
                     beta: Optional[Sequence[float]] = None, r: Sequence[float] = R_NONE,
                     tau: float = 1e-3, steps: int = 4, scheme: str = "l2b", q: int = 4,
                     lam: float = 1.0) -> Problem:
    """Constant diffusion a == a_const; u0 a seeded sine series (not normalised).

    Returns the problem and leaves the sine coefficients recoverable through
    ``sine_coefficients`` with the same seed.
    """
    n = tuple(int(m) for m in n)
    d = len(n)
    rng = np.random.default_rng(seed)
    s_u = sine_series(rng, n, [u_kmax] * d, include_boundary=False)
    a = np.full(tuple(m + 2 for m in reversed(n)), float(a_const))
    return Problem(d=d, n=n, a=a, u0=np.ascontiguousarray(s_u),
                   beta=tuple(beta) if beta is not None else (0.0,) * d,
                   r=tuple(float(x) for x in r), tau=tau, steps=steps, scheme=scheme, q=q,
                   lam=lam)


def sine_coefficients(n: Sequence[int], seed: int, u_kmax: int) -> np.ndarray:
    """The coefficient array c[k_d..k_1] that ``constant_problem`` drew for u0."""
    d = len(n)
    rng = np.random.default_rng(seed)
    kshape = (u_kmax,) * d
    grids = np.meshgrid(*[np.arange(1, u_kmax + 1) for _ in range(d)], indexing="ij")
    ksq = sum(g.astype(np.float64) ** 2 for g in grids)
    return rng.standard_normal(kshape) / ksq


# --------------------------------------------------------------------------
# Named workloads. T = 0.1 everywhere, tau = T/steps.
# --------------------------------------------------------------------------

def workload(name: str, seed: int = 0) -> Problem:
    """The named synthetic workloads (2D 63^2 LE; 3D 127^3; 3D 255^3; 3D 383^3)."""
    if name == "2d_n63_le":
        return smooth_problem((63, 63), seed, a_amp=0.5, a_kmax=4, u_kmax=8, beta=(0.5, 0.5),
                              r=R_LOGISTIC, tau=1e-3, steps=100, scheme="le", name=name)
    if name == "3d_n127_l2b":
        return smooth_problem((127,) * 3, seed, a_amp=0.9, beta=(10.0,) * 3, r=R_CUBIC,
                              tau=5e-4, steps=200, scheme="l2b", name=name)
    if name == "3d_n127_etd2rk":
        return smooth_problem((127,) * 3, seed, a_amp=0.9, beta=(10.0,) * 3, r=R_CUBIC,
                              tau=5e-4, steps=200, scheme="etd2rk", q=4, name=name)
    if name == "3d_n255_l2b":
        return smooth_problem((255,) * 3, seed, a_amp=0.9, beta=(10.0,) * 3, r=R_CUBIC,
                              tau=1e-3, steps=100, scheme="l2b", name=name)
    if name == "3d_n383_etd2rk":
        return anisotropic_problem(383, seed, tau=2e-3, steps=50, scheme="etd2rk", q=6, name=name)
    # the same ETD2RK workloads with exact phi1 (q = 0: no quadrature nodes)
    if name == "3d_n127_etd2rk_exact":
        return smooth_problem((127,) * 3, seed, a_amp=0.9, beta=(10.0,) * 3, r=R_CUBIC,
                              tau=5e-4, steps=200, scheme="etd2rk", q=0, name=name)
    if name == "3d_n383_etd2rk_exact":
        return anisotropic_problem(383, seed, tau=2e-3, steps=50, scheme="etd2rk", q=0, name=name)
    # the paper's own 3D problem at the size of its timing runs (Sec. 5.2: N = 60, b = -0.01,
    # SL2 with the lambda of Table tab:adr3d_lambdaopt, m = 2^8 steps to T = 1/4)
    if name == "3d_paper_n60_sl2":
        return paper3d_problem(60, -0.01, 0.53, scheme="sl2", steps=256, name=name)
    if name == "2d_paper_n256_sl2":
        return paper2d_problem(256, 0.57, scheme="sl2", steps=256, name=name)
    raise KeyError(name)


def paper3d_problem(N: int, b: float, lam: float, *, scheme: str = "l2b", steps: int = 256, T: float = 0.25,
                    name: str = "") -> Problem:
    """The three-dimensional problem of Sec. 5.2, eq. (eq:adr3d), split as eq. (eq:adr3dstab):
    u_t = a Lap u + b (d_1 + d_2 + d_3) u + u(1 + u^2) on (0,1)^3, Dirichlet data on the faces
    x_mu = 0, homogeneous Neumann data on x_mu = 1, a = exp(-|x - 1/2|^2)/10,
    u0 = (27/4)^3 prod x_mu (1 - x_mu)^2, N points per direction (x_i = i/N), the whole
    advection in the extracted operator (beta_bar = beta)."""
    h = 1.0 / N
    x = h * np.arange(1, N + 1)
    xa = h * np.arange(0, N + 2)
    xa[N + 1] = xa[N - 1] if N >= 2 else 0.0        # mirror node beyond the Neumann face
    g1 = np.exp(-(xa - 0.5) ** 2)
    a = 0.1 * g1[:, None, None] * g1[None, :, None] * g1[None, None, :]
    f = x * (1.0 - x) ** 2
    u0 = (27.0 / 4.0) ** 3 * f[:, None, None] * f[None, :, None] * f[None, None, :]
    return Problem(d=3, n=(N, N, N), a=a, u0=u0, beta=(b, b, b), r=(0.0, 1.0, 0.0, 1.0), tau=T / steps,
                   steps=steps, scheme=scheme, lam=lam, beta_bar=(b, b, b), bc=(1, 1, 1), form="nondiv",
                   name=name or f"paper3d_N{N}")


PERIODIC = 2


def paper2d_problem(N: int, lam: float, *, scheme: str = "l2b", steps: int = 256, T: float = 4.0,
                    name: str = "") -> Problem:
    """The two-dimensional problem of Sec. 5.1, eq. (eq:ad2d): periodic on (-3 pi, 3 pi)^2,
    diffusion tensor diag(1/2 + sin^2 x1 sin^2 x2 / 6, 1/2 + cos^2 x1 cos^2 x2 / 6), velocity
    b = (sin^2 x1, sin^2 x2)/5 in div(b u), r(u) = u(1 - u)/4, u0 = exp(-(x1^2 + x2^2)),
    N points per direction. The extracted velocity of eq. (eq:amaxbeta) is the mean of
    b_mu + d_mu a_mumu over the box, 1/10 on both axes (the derivative term has mean zero)."""
    L = 6.0 * np.pi
    x = -3.0 * np.pi + L / N * np.arange(N)
    X2, X1 = np.meshgrid(x, x, indexing="ij")           # arrays [x2][x1]
    a = np.stack([0.5 + np.sin(X1) ** 2 * np.sin(X2) ** 2 / 6.0, 0.5 + np.cos(X1) ** 2 * np.cos(X2) ** 2 / 6.0])
    vel = np.stack([np.sin(X1) ** 2 / 5.0, np.sin(X2) ** 2 / 5.0])
    u0 = np.exp(-(X1 ** 2 + X2 ** 2))
    return Problem(d=2, n=(N, N), a=a, u0=u0, beta=(0.1, 0.1), r=(0.0, 0.25, -0.25, 0.0), tau=T / steps,
                   steps=steps, scheme=scheme, lam=lam, beta_bar=(0.1, 0.1), bc=(PERIODIC, PERIODIC), form="flux",
                   length=(L, L), velocity=vel, name=name or f"paper2d_N{N}")


def paper1d_problem(N: int, lam: float, *, nonlinear: bool, scheme: str = "l2b", steps: int = 256,
                    T: Optional[float] = None, name: str = "") -> Problem:
    """The one-dimensional periodic problems of Sec. 4 on (-pi, pi) with
    a = 1 + 10 sin^2 x (a_max over the grid = 11 for N divisible by 4), u0 = sin x:
    eq. (eq:adlinearzero) u_t = a u_xx (nonlinear = False, T = 1/40) or eq. (eq:adnonlinear)
    u_t = (a u_x)_x + u(1 - u) (nonlinear = True, T = 1/10). Stored as a 2D periodic
    problem with one point along x2 (whose derivatives vanish)."""
    if T is None:
        T = 0.1 if nonlinear else 1.0 / 40.0
    L = 2.0 * np.pi
    x = -np.pi + L / N * np.arange(N)
    a1 = 1.0 + 10.0 * np.sin(x) ** 2
    a = np.stack([a1[None, :], np.ones((1, N))])
    u0 = np.sin(x)[None, :]
    r = (0.0, 1.0, -1.0, 0.0) if nonlinear else (0.0, 0.0, 0.0, 0.0)
    return Problem(d=2, n=(N, 1), a=a, u0=u0, beta=(0.0, 0.0), r=r, tau=T / steps, steps=steps, scheme=scheme,
                   lam=lam, beta_bar=(0.0, 0.0), bc=(PERIODIC, PERIODIC), form="flux" if nonlinear else "nondiv",
                   length=(L, L), velocity=None, name=name or f"paper1d_N{N}")


WORKLOADS = ("2d_n63_le", "3d_n127_l2b", "3d_n127_etd2rk", "3d_n255_l2b", "3d_n383_etd2rk",
             "3d_n127_etd2rk_exact", "3d_n383_etd2rk_exact", "3d_paper_n60_sl2", "2d_paper_n256_sl2")


# --------------------------------------------------------------------------
# Served stream: 512 solves, Poisson arrivals at 200/s.
# --------------------------------------------------------------------------

@dataclass
class StreamRequest:
    index: int
    arrival_s: float
    d: int
    n: int
    beta: Tuple[float, ...]
    r: Tuple[float, float, float, float]
    steps: int
    seed: int

    def problem(self) -> Problem:
        tau = 0.1 / self.steps
        return smooth_problem((self.n,) * self.d, self.seed, a_amp=0.9, beta=self.beta, r=self.r,
                              tau=tau, steps=self.steps, scheme="l2b",
                              name=f"req{self.index}_{self.d}d_n{self.n}")


def request_stream(count: int = 512, seed: int = 1, rate_hz: float = 200.0,
                   sizes_2d: Sequence[int] = (63, 127, 255, 511),
                   sizes_3d: Sequence[int] = (31, 63, 127, 191),
                   steps_range: Tuple[int, int] = (20, 200)) -> List[StreamRequest]:
    """Seeded request stream: exponential inter-arrivals, fair coins for d and f."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        d = 2 if rng.random() < 0.5 else 3
        n = int(rng.choice(sizes_2d if d == 2 else sizes_3d))
        beta = tuple(float(b) for b in rng.uniform(0.0, 20.0, size=d))
        r = R_LOGISTIC if rng.random() < 0.5 else R_CUBIC
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append(StreamRequest(index=i, arrival_s=t, d=d, n=n, beta=beta, r=r, steps=steps,
                                 seed=1000 + i))
    return out
