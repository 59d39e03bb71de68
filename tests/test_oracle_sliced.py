"""Pins of the exact-slice oracle (oracle/sliced.py) against facts that do not depend
on it: exact integer arithmetic, a pure-Python evaluation of the definition, exact
products for small-integer data, and the 2^(-8S) error bound with its decay in S."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import adr, expo, sliced


def py_digits(x: float, e: int, S: int):
    """Balanced base-256 digits of x by exact integer arithmetic (MSB first)."""
    Y = round(Fraction(x) * Fraction(2) ** (8 * S - 1 - e))     # halves to even
    Y0 = Y
    ds = []
    for _ in range(S):
        b = (Y + 128) % 256 - 128
        ds.append(b)
        Y = (Y - b) // 256
    assert Y == 0
    return ds[::-1], Y0


def py_exponent(row):
    """The least e with m (1 + 2^-7) < 2^e, m the row maximum and the product rounded to
    FP64 (Python floats multiply in IEEE double)."""
    m = float(max(abs(v) for v in row)) * (1.0 + 2.0 ** -7)
    if m == 0:
        return 0
    e = 0
    while Fraction(m) >= Fraction(2) ** e:
        e += 1
    while Fraction(m) < Fraction(2) ** (e - 1):
        e -= 1
    return e


@pytest.mark.parametrize("S", [3, 4, 5, 6, 7])
def test_digits_round_trip_exact(S):
    rng = np.random.default_rng(S)
    X = rng.standard_normal((5, 9)) * np.exp(rng.uniform(-20, 20, (5, 1)))
    X[1, 3] = 0.0
    X[2] = 0.0
    X[3, 4] = -np.max(np.abs(X[3]))                 # the row maximum with a negative sign
    # maxima just below a power of two: 0.99 keeps e = 0 (Y near the top of the digit
    # range), 0.9999 is lifted to e = 1 by the 1 + 2^-7 margin
    X[0] *= 0.99 / np.max(np.abs(X[0]))
    X[4] *= 0.9999 / np.max(np.abs(X[4]))
    e = sliced.exponents(X)
    assert (e[0], e[4]) == (0, 1)
    D = sliced.digits(X, e, S)
    assert np.all(D >= -128) and np.all(D <= 127)
    for i in range(X.shape[0]):
        assert e[i] == py_exponent(X[i])
        for k in range(X.shape[1]):
            ds, Y = py_digits(X[i, k], int(e[i]), S)
            assert [int(D[s, i, k]) for s in range(S)] == ds
            # the digits represent x to half a unit of the last digit
            rep = sum(Fraction(d) * Fraction(256) ** (S - 1 - s) for s, d in enumerate(ds))
            assert rep == Y
            # within the positive range of S balanced digits
            assert -Fraction(128 * (256 ** S - 1), 255) <= Y <= Fraction(127 * (256 ** S - 1), 255)
            err = abs(rep * Fraction(2) ** (int(e[i]) + 1 - 8 * S) - Fraction(X[i, k]))
            assert err <= Fraction(2) ** (int(e[i]) - 8 * S)


def py_matmul_rows(A, B, S):
    """The definition evaluated with Python integers and fractions, then rounded."""
    out = np.empty((A.shape[0], B.shape[0]))
    for i in range(A.shape[0]):
        a = py_exponent(A[i])
        fa = [py_digits(v, a, S)[0] for v in A[i]]
        for j in range(B.shape[0]):
            b = py_exponent(B[j])
            fb = [py_digits(v, b, S)[0] for v in B[j]]
            P = [0] * S
            for s in range(S):
                for t in range(S - s):
                    P[s + t] += sum(fa[k][s] * fb[k][t] for k in range(A.shape[1]))
            # top level down, one rounding per level as in FP64
            v = float(P[S - 1])
            for lvl in range(S - 2, -1, -1):
                v = v * 2.0 ** -8 + float(P[lvl])
            out[i, j] = np.ldexp(v, a + b - 14)
    return out


@pytest.mark.parametrize("S", [3, 4, 6, 7])
def test_matmul_matches_pure_python_definition(S):
    rng = np.random.default_rng(10 + S)
    A = rng.standard_normal((4, 11)) * np.array([[1.0], [1e-3], [3e5], [0.5]])
    B = rng.standard_normal((3, 11))
    B[1, :5] = 0.0
    assert np.array_equal(sliced.matmul_rows(A, B, S), py_matmul_rows(A, B, S))


def test_small_integers_are_exact():
    """Rows of integers |x| <= 127 (max 127, e = 8 since 127 (1 + 2^-7) = 128) are exact
    in the top two digits (Y = x 2^(8S-9)), so every product falls in levels s + t <= 2 < S
    and the result is the exact integer product."""
    rng = np.random.default_rng(3)
    A = rng.integers(-127, 128, (6, 40)).astype(float)
    B = rng.integers(-127, 128, (7, 40)).astype(float)
    A[:, 0] = 127.0
    B[:, 0] = -127.0
    for S in (3, 5, 7):
        assert np.array_equal(sliced.matmul_rows(A, B, S), A @ B.T)


def test_error_bound_and_decay():
    """|C - A B^T| <= 2^(-8S) * 16 S * K * max|A_i| max|B_j| (each value is within
    2^(e-8S) <= 2.02 2^(-8S) max of its digits, and the first dropped level holds S - 1
    products of at most 2^14 * 2^(a+b+2-8S-16)), and each extra digit gains about 2^8."""
    rng = np.random.default_rng(4)
    K = 200
    A = rng.standard_normal((20, K))
    B = rng.standard_normal((30, K))
    ref = A @ B.T
    scale = np.max(np.abs(A), axis=1)[:, None] * np.max(np.abs(B), axis=1)[None, :]
    errs = {}
    for S in range(3, 8):
        err = np.abs(sliced.matmul_rows(A, B, S) - ref)
        assert np.all(err <= 2.0 ** (-8 * S) * 16 * S * K * scale + 1e-13 * np.abs(ref).max())
        errs[S] = float(np.max(err / scale))
    for S in range(3, 6):
        assert 2 ** 5 < errs[S] / errs[S + 1] < 2 ** 11, errs


def test_sliced_action_within_bound():
    """Three sliced mode products vs the exact exponential action (heat-kernel factors:
    rows of |E| sum to at most 1)."""
    p = synth.smooth_problem((17, 13, 11), 5, tau=2e-3)
    op = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau)
    V = np.random.default_rng(5).standard_normal(p.shape)
    ref = op.expv(1.0, V)
    mats = op.factors(1.0)
    K = max(p.n)
    emax = max(float(np.max(np.abs(M))) for M in mats)
    for S in (3, 5, 7):
        got = sliced.tucker(V, mats, S)
        bound = 3 * 2.0 ** (-8 * S) * 16 * S * K * emax * np.max(np.abs(V))
        assert np.max(np.abs(got - ref)) <= bound + 1e-14 * np.max(np.abs(V))


def test_sliced_solve_converges_to_fp64_solve():
    p = synth.smooth_problem((12, 10, 9), 6, tau=1e-3, steps=5, scheme="l2b")
    from oracle import schemes as Sch
    ref = Sch.solve(p)
    e4 = np.max(np.abs(sliced.solve(p, 4) - ref))
    e7 = np.max(np.abs(sliced.solve(p, 7) - ref))
    assert e7 < 1e-12 * np.max(np.abs(ref))
    assert e7 < e4
