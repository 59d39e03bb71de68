"""Pins of the exact-slice oracle (oracle/sliced.py) against facts that do not depend
on it: exact integer arithmetic, a pure-Python evaluation of the definition, exact
products for 7-bit integer data, and the 2^(-7S) error bound with its decay in S."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import adr, expo, sliced


def py_digits(x: float, e: int, S: int):
    """Digits of x by exact rational arithmetic (round half to even)."""
    y = Fraction(abs(x)) * Fraction(2) ** (7 * S - e)
    Y = round(y)                       # Python rounds halves to even
    Y = min(Y, 2 ** (7 * S) - 1)
    ds = []
    for s in range(S):
        p = S - 1 - s
        ds.append((Y // 128 ** p) % 128)
    sgn = -1 if x < 0 else 1
    return [sgn * d for d in ds], Y


def py_exponent(row):
    m = max(abs(v) for v in row)
    if m == 0:
        return 0
    e = 0
    while Fraction(m) >= Fraction(2) ** e:
        e += 1
    while Fraction(m) < Fraction(2) ** (e - 1):
        e -= 1
    return e


@pytest.mark.parametrize("S", [3, 5, 7, 8])
def test_digits_round_trip_exact(S):
    rng = np.random.default_rng(S)
    X = rng.standard_normal((5, 9)) * np.exp(rng.uniform(-20, 20, (5, 1)))
    X[1, 3] = 0.0
    X[2] = 0.0
    e = sliced.exponents(X)
    D = sliced.digits(X, e, S)
    for i in range(X.shape[0]):
        assert e[i] == py_exponent(X[i])
        for k in range(X.shape[1]):
            ds, Y = py_digits(X[i, k], int(e[i]), S)
            assert [int(D[s, i, k]) for s in range(S)] == ds
            # the digits represent x to half a unit of the last digit
            rep = sum(Fraction(d) * Fraction(128) ** (S - 1 - s) for s, d in enumerate(ds))
            err = abs(rep * Fraction(2) ** (int(e[i]) - 7 * S) - Fraction(X[i, k]))
            assert err <= Fraction(2) ** (int(e[i]) - 7 * S - 1) + Fraction(2) ** (int(e[i]) - 7 * S) * (Y == 2 ** (7 * S) - 1)


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
                v = v * 2.0 ** -7 + float(P[lvl])
            out[i, j] = np.ldexp(v, a + b - 14)
    return out


@pytest.mark.parametrize("S", [3, 4, 6, 8])
def test_matmul_matches_pure_python_definition(S):
    rng = np.random.default_rng(10 + S)
    A = rng.standard_normal((4, 11)) * np.array([[1.0], [1e-3], [3e5], [0.5]])
    B = rng.standard_normal((3, 11))
    B[1, :5] = 0.0
    assert np.array_equal(sliced.matmul_rows(A, B, S), py_matmul_rows(A, B, S))


def test_seven_bit_integers_are_exact():
    """Rows whose entries are integers |x| <= 127 with max 127 have one nonzero digit:
    only level 0 survives and the product is the exact integer product."""
    rng = np.random.default_rng(3)
    A = rng.integers(-127, 128, (6, 40)).astype(float)
    B = rng.integers(-127, 128, (7, 40)).astype(float)
    A[:, 0] = 127.0
    B[:, 0] = -127.0
    for S in (3, 5, 8):
        assert np.array_equal(sliced.matmul_rows(A, B, S), A @ B.T)


def test_error_bound_and_decay():
    """|C - A B^T| <= 2^(-7S) * 4 S * K * max|A_i| max|B_j|, and each extra digit gains
    about 2^7."""
    rng = np.random.default_rng(4)
    K = 200
    A = rng.standard_normal((20, K))
    B = rng.standard_normal((30, K))
    ref = A @ B.T
    scale = np.max(np.abs(A), axis=1)[:, None] * np.max(np.abs(B), axis=1)[None, :]
    errs = {}
    for S in range(3, 9):
        err = np.abs(sliced.matmul_rows(A, B, S) - ref)
        assert np.all(err <= 2.0 ** (-7 * S) * 4 * S * K * scale + 1e-13 * np.abs(ref).max())
        errs[S] = float(np.max(err / scale))
    for S in range(3, 6):
        assert 2 ** 4 < errs[S] / errs[S + 1] < 2 ** 10, errs


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
        bound = 3 * 2.0 ** (-7 * S) * 4 * S * K * emax * np.max(np.abs(V))
        assert np.max(np.abs(got - ref)) <= bound + 1e-14 * np.max(np.abs(V))


def test_sliced_solve_converges_to_fp64_solve():
    p = synth.smooth_problem((12, 10, 9), 6, tau=1e-3, steps=5, scheme="l2b")
    from oracle import schemes as Sch
    ref = Sch.solve(p)
    e5 = np.max(np.abs(sliced.solve(p, 5) - ref))
    e8 = np.max(np.abs(sliced.solve(p, 8) - ref))
    assert e8 < 1e-12 * np.max(np.abs(ref))
    assert e8 < e5
