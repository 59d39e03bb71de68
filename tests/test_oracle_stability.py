"""Pin: the stability functions of Sec. 2 give the lower bounds of Table tab:stab."""
import numpy as np
import pytest

from oracle import stability as St

TABLE = {  # Table tab:stab, lower bound on lam for unconditional stability
    "ee": 0.5, "erk2p2": 0.5, "erk2p1": 1.0 / 3.0, "l2a": 0.301, "l2b": 0.301,
    "le": 0.218, "sle": 1.0 / (2.0 * np.e), "sl2": 0.183,
}


@pytest.mark.parametrize("scheme", sorted(TABLE))
def test_table_bound(scheme):
    b = St.stability_bound(St.PHI[scheme])
    assert b is not None
    # the table prints three digits; exact values are stated for ee, erk2p*, sle
    assert abs(b - TABLE[scheme]) < 1.5e-3, b


def test_lawson_euler_root():
    """Theorem thm:lawsoneuler: the bound is the zero of 1 - 1/lam + exp(1/(1-lam))."""
    from scipy.optimize import brentq
    root = brentq(lambda l: 1 - 1 / l + np.exp(1 / (1 - l)), 0.1, 0.5)
    assert abs(root - St.stability_bound(St.PHI["le"])) < 1e-4


def test_quadrature_forms_never_amplify_at_lam_one():
    z = -np.geomspace(1e-4, 1e5, 4000)
    for q in (4, 6):
        assert np.max(np.abs(St.phi_etd2rk_quad(z, 1.0, q))) <= 1.0 + 1e-12
        assert np.max(np.abs(St.phi_erk2p1f_quad(z, 1.0, q))) <= 1.0 + 1e-12
    # the e^{tau A} u form damps the stiff end, the Appendix form leaves it at 1
    assert abs(St.phi_etd2rk_quad(np.array([-1e5]), 1.0, 4)[0]) < 1e-3
    assert abs(abs(St.phi_erk2p1f_quad(np.array([-1e5]), 1.0, 4)[0]) - 1.0) < 1e-3
