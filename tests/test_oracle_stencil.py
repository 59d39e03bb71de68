"""Pins for the oracle's remainder g(u) and right-hand side F(u) (eq:nonlin, Sec. 5.2)."""
import numpy as np
import pytest

import synth
from oracle import adr


def _grid(n):
    return [np.arange(1, m + 1) / (m + 1) for m in n]


def _nodes(n):
    return [np.arange(0, m + 2) / (m + 1) for m in n]


def _outer(vecs):
    """C-ordered product field from per-axis vectors listed x1 first."""
    out = np.ones(1)
    for v in reversed(vecs):
        out = np.multiply.outer(out, v)
    return out.reshape(tuple(len(v) for v in reversed(vecs)))


def _laplacian_loops(u, hs):
    """plain-loop 5/7-point Laplacian with zero Dirichlet ghosts (independent of adr)."""
    d = u.ndim
    out = np.zeros_like(u)
    for idx in np.ndindex(*u.shape):
        s = 0.0
        for mu in range(d):
            ax = d - 1 - mu
            up = list(idx); up[ax] += 1
            dn = list(idx); dn[ax] -= 1
            vu = u[tuple(up)] if up[ax] < u.shape[ax] else 0.0
            vd = u[tuple(dn)] if dn[ax] >= 0 else 0.0
            s += (vu - 2 * u[idx] + vd) / hs[mu] ** 2
        out[idx] = s
    return out


@pytest.mark.parametrize("n", [(6, 5), (5, 4, 3)])
def test_constant_a_reduces_to_scaled_laplacian(n):
    rng = np.random.default_rng(1)
    u = rng.standard_normal(tuple(reversed(n)))
    a = np.full(tuple(m + 2 for m in reversed(n)), 1.3)
    lam = 0.6
    g = adr.remainder(u, a, (0.0,) * len(n), synth.R_NONE, lam, (0.0,) * len(n), 1.3)
    ref = (1.3 - lam * 1.3) * _laplacian_loops(u, adr.mesh_widths(n))
    assert np.max(np.abs(g - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [(9, 8), (7, 6, 5)])
def test_quadratic_fields_are_exact(n):
    """u = prod x(1-x) (zero on the boundary), a linear in x: the flux form with
    mean face values differentiates (a u')' exactly, centred differences give u' exactly."""
    d = len(n)
    xs, nodes = _grid(n), _nodes(n)
    coef = [1.0, 2.0, -0.5][:d]
    fac = [x * (1 - x) for x in xs]
    u = _outer(fac)
    # a = 1 + sum coef_mu x_mu on all nodes
    a = 1.0 + sum(coef[mu] * _outer([nodes[nu] if nu == mu else np.ones_like(nodes[nu]) for nu in range(d)])
                  for mu in range(d))
    beta = (0.7, -1.1, 2.0)[:d]
    r = (0.1, -0.3, 0.2, 0.05)
    F = adr.full_rhs(u, a, beta, r)
    # exact continuous value at the interior nodes
    ai = 1.0 + sum(coef[mu] * _outer([xs[nu] if nu == mu else np.ones_like(xs[nu]) for nu in range(d)])
                   for mu in range(d))
    ref = r[0] + r[1] * u + r[2] * u ** 2 + r[3] * u ** 3
    for mu in range(d):
        d1 = _outer([(1 - 2 * xs[nu]) if nu == mu else fac[nu] for nu in range(d)])
        d2 = _outer([(-2.0 * np.ones_like(xs[nu])) if nu == mu else fac[nu] for nu in range(d)])
        ref = ref + coef[mu] * d1 + ai * d2 + beta[mu] * d1
    assert np.max(np.abs(F - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_split_identity_F_equals_Au_plus_g():
    """F(u) = (A_d (+) .. (+) A_1) u + g(u) for the extracted A of eq:linop."""
    p = synth.smooth_problem((11, 9, 8), 2, lam=0.7, beta_bar=(3.0, -1.0, 0.5))
    amax = adr.extracted_amax(p.a)
    mats = [adr.operator_1d(p.n[mu], amax, p.lam, p.beta_bar[mu]) for mu in range(3)]
    g = adr.remainder(p.u0, p.a, p.beta, p.r, p.lam, p.beta_bar, amax)
    F = adr.full_rhs(p.u0, p.a, p.beta, p.r)
    assert np.max(np.abs(F - adr.apply_kron_sum(p.u0, mats) - g)) <= 1e-12 * np.max(np.abs(F))


def test_second_order_consistency():
    """manufactured smooth u, a: F(u) -> div(a grad u) + beta.grad u + r(u) at O(h^2)."""
    errs = []
    beta = (1.5, -0.5)
    r = (0.0, 1.0, -1.0, 0.0)
    for m in (15, 31, 63):
        n = (m, m)
        xs, nodes = _grid(n), _nodes(n)
        X2, X1 = np.meshgrid(xs[1], xs[0], indexing="ij")
        N2, N1 = np.meshgrid(nodes[1], nodes[0], indexing="ij")
        u = np.sin(np.pi * X1) * np.sin(2 * np.pi * X2)
        af = lambda x1, x2: 1.0 + 0.5 * np.cos(x1 + 2 * x2)
        a = af(N1, N2)
        F = adr.full_rhs(u, a, beta, r)
        ux1 = np.pi * np.cos(np.pi * X1) * np.sin(2 * np.pi * X2)
        ux2 = 2 * np.pi * np.sin(np.pi * X1) * np.cos(2 * np.pi * X2)
        lap = -(np.pi ** 2 + 4 * np.pi ** 2) * u
        ax1 = -0.5 * np.sin(X1 + 2 * X2)
        ax2 = -1.0 * np.sin(X1 + 2 * X2)
        ref = af(X1, X2) * lap + ax1 * ux1 + ax2 * ux2 + beta[0] * ux1 + beta[1] * ux2 + u - u ** 2
        errs.append(np.max(np.abs(F - ref)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.1), orders


def test_amax_includes_boundary_nodes():
    a = np.ones((5, 6))
    a[0, 3] = 4.0
    assert adr.extracted_amax(a) == 4.0
