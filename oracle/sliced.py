"""Exact-slice contractions, written from their definition (oracle; test infrastructure
only: tests and the benchmark's CPU baseline use it, the product path never does).

The sliced precision is not from the paper; it is an error-free splitting of the
operands in the manner of Ozaki, Ogita, Oishi and Rump (Numer. Algorithms 59, 2012),
used here to run the mu-mode products on integer matrix units.

Definition (S digits, 3 <= S <= 7).
  * Every factor row and every fiber of the grid operand (the values along the
    contracted axis with all other indices fixed) gets the exponent e with
    m (1 + 2^-7) < 2^e for its maximum m = max|x| (the frexp exponent of the FP64
    product m * (1 + 2^-7); e = 0 for an all-zero row), so that max|x| < 0.993 2^e.
  * A value x becomes the integer Y = round_half_even(x 2^(8S - 1 - e)), so that
    |Y| < 0.4963 256^S, written in balanced base 256: Y = sum_(i<S) b_i 256^i with
    every b_i in [-128, 127] (unique; S balanced digits cover [-0.502, 0.498] 256^S,
    so every such Y has one). Digit planes are kept most significant first,
    d_s = b_(S-1-s), so that
        x ~ 2^(e+1) sum_s d_s 2^(-8(s+1)).
  * A factor row (exponent a, digits f_s) contracted with a fiber (exponent b,
    digits v_t) keeps the digit products with s + t < S:
        sum_k f v ~ 2^(a + b - 14) sum_(l<S) 2^(-8 l) P_l,
        P_l = sum_(s+t=l) sum_k f_s[k] v_t[k]      (exact integers),
    combined from the top level down, v <- v 2^-8 + P_l, in FP64.
The errors are the dropped levels s + t >= S and the rounding of Y, both of order
2^(-8S) relative to the row and fiber scales.

Pins: tests/test_oracle_sliced.py (digit expansion against exact integer arithmetic,
exactness for small-integer data, a pure-Python evaluation of the definition on small
cases, the 2^(-8S) error bound and its decay with S).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .expo import axis_of


def exponents(X: np.ndarray) -> np.ndarray:
    """e with max|x| (1 + 2^-7) < 2^e along the last axis (0 for all-zero rows)."""
    mx = np.max(np.abs(X), axis=-1)
    _, e = np.frexp(mx * (1.0 + 2.0 ** -7))
    return e.astype(np.int64)


def digits(X: np.ndarray, e: np.ndarray, S: int) -> np.ndarray:
    """Balanced base-256 digits (S, *X.shape), most significant first, of X relative to
    row exponents e (X.shape[:-1])."""
    Y = np.rint(np.ldexp(X, (8 * S - 1 - e)[..., None])).astype(np.int64)
    out = np.empty((S,) + X.shape)
    for i in range(S):                          # least significant first
        b = ((Y + 128) & 255) - 128
        out[S - 1 - i] = b
        Y = (Y - b) >> 8
    assert not np.any(Y), "digit expansion did not terminate"
    return out


def matmul_rows(A: np.ndarray, B: np.ndarray, S: int) -> np.ndarray:
    """C[i, j] = sum_k A[i, k] B[j, k] by the sliced definition (rows of A and B scaled
    separately). Integer-valued FP64 products are exact: every partial sum is far below
    2^53."""
    ea, eb = exponents(A), exponents(B)
    da, db = digits(A, ea, S), digits(B, eb, S)
    P = [np.zeros((A.shape[0], B.shape[0])) for _ in range(S)]
    for s in range(S):
        for t in range(S - s):
            P[s + t] += da[s] @ db[t].T
    v = P[S - 1]
    for lvl in range(S - 2, -1, -1):
        v = v * 2.0 ** -8 + P[lvl]
    return np.ldexp(v, ea[:, None] + eb[None, :] - 14)


def mode_product(V: np.ndarray, M: np.ndarray, mu: int, S: int) -> np.ndarray:
    """Sliced V x_mu M: contract spatial index mu (x1 = 0) of V with the columns of M."""
    ax = axis_of(mu, V.ndim)
    W = np.moveaxis(V, ax, -1)
    lead = W.shape[:-1]
    C = matmul_rows(M, W.reshape(-1, W.shape[-1]), S)          # (n_out, fibers)
    C = C.reshape((M.shape[0],) + lead)
    return np.ascontiguousarray(np.moveaxis(C, 0, ax))


def tucker(V: np.ndarray, mats: Sequence[np.ndarray], S: int) -> np.ndarray:
    """Sliced V x_1 M_1 x_2 M_2 (x_3 M_3), modes in the order 1, 2, 3."""
    W = V
    for mu, M in enumerate(mats):
        W = mode_product(W, M, mu, S)
    return W


class SlicedBackend:
    """Grid backend of the Lawson schemes whose exponential actions are sliced
    mu-mode products (the remainder and F stay FP64)."""

    def __init__(self, prob, S: int):
        from .schemes import GridBackend
        self._fp64 = GridBackend(prob)
        self.op = self._fp64.op
        self.S = S

    def expv(self, c, v):
        return tucker(v, self.op.factors(c), self.S)

    def g(self, v):
        return self._fp64.g(v)

    def F(self, v):
        return self._fp64.F(v)


def solve(prob, S: int, steps=None) -> np.ndarray:
    """The problem's Lawson scheme with sliced exponential actions."""
    from .schemes import integrate
    if prob.scheme not in ("le", "l2b", "sle", "l2a", "sl2"):
        raise ValueError("the sliced oracle covers the Lawson schemes (only exponential actions)")
    be = SlicedBackend(prob, S)
    return integrate(prob.u0, be, prob.tau, prob.steps if steps is None else steps, prob.scheme)
