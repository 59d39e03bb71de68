"""Pin: the oracle's step code reproduces the errors printed in Sec. 4.1,
Figure fig:ad1dex0_diffdeltaa (1D linear diffusion, Fourier, lam = 1, 1/2, 1/3).

The reference is the exact semi-discrete solution (the paper measures against
the exact solution); the printed errors carry about 2e-12 absolute error of the
paper's own reference, so the bar is 1e-6 relative plus 5e-12 absolute. The
exponential Euler series carries a constant offset of about 4e-11 (lam = 1/2 and
1/3) or 4e-12 (lam = 1) at every m, the same at m = 16 as at m = 1024, so it
comes from the paper's evaluation of phi1, not from the step; its bar is 5e-11.
"""
import os

import numpy as np
import pytest

from oracle import fourier1d as F1
from oracle import schemes as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_linear_diffusion_errors.txt")
LAM = {"1": 1.0, "1/2": 0.5, "1/3": 1.0 / 3.0}


def _rows(max_m):
    out = []
    for ln in open(GOLD):
        if ln.startswith("#") or not ln.strip():
            continue
        lam, sch, m, err = ln.split()
        if int(m) <= max_m:
            out.append((lam, sch, int(m), float(err)))
    return out


@pytest.fixture(scope="module")
def reference():
    N, T = 4096, 1.0 / 40.0
    x = -np.pi + 2.0 * np.pi * np.arange(N) / N
    return x, F1.exact_solution(x, T)


def test_fixture_complete():
    rows = _rows(16384)
    assert len(rows) == 134
    # every scheme has the lam = 1 and lam = 1/2 panels at six step counts
    for lam in ("1", "1/2"):
        for sch in ("sle", "le", "ee", "erk2p2", "sl2", "erk2p1", "l2a", "l2b"):
            assert len([r for r in rows if r[0] == lam and r[1] == sch]) == 6


@pytest.mark.parametrize("row", _rows(1024), ids=lambda r: f"{r[0]}-{r[1]}-{r[2]}")
def test_printed_error(reference, row):
    lam, sch, m, printed = row
    x, ref = reference
    T = 1.0 / 40.0
    be = F1.Fourier1D(4096, LAM[lam], T / m)
    u = S.integrate(np.sin(x), be, T / m, m, sch)
    err = S.rel_inf_error(u, ref)
    absolute = 5e-11 if sch == "ee" else 5e-12
    assert abs(err - printed) <= 1e-6 * printed + absolute, (err, printed)


def test_exact_reference_is_the_semi_discrete_solution(reference):
    """L2b errors against the Galerkin reference fall by 4 per halving of tau
    (second order); an error of the reference above ~1e-10 would break the ratio."""
    x, ref = reference
    T = 1.0 / 40.0
    errs = []
    for m in (4096, 8192):
        be = F1.Fourier1D(4096, 1.0, T / m)
        errs.append(S.rel_inf_error(S.integrate(np.sin(x), be, T / m, m, "l2b"), ref))
    assert 3.95 < errs[0] / errs[1] < 4.05, errs
