"""Brute-force forms of the Kronecker-sum operations (oracle; test infrastructure only).

Sec. 1: the vec of a tensor V (x1 fastest) is the C-order ravel of the numpy
array of shape (n_d, ..., n_1). With that ordering the Kronecker sum
A_d (+) ... (+) A_1 is sum_mu I (x) .. (x) A_mu (x) .. (x) I with A_mu in the
slot of axis mu counted from the slowest axis. These dense forms are only for
grids with a few hundred unknowns.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def kron_sum(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Dense A_d (+) ... (+) A_1 for mats = [A_1, ..., A_d]."""
    d = len(mats)
    sizes = [M.shape[0] for M in mats]
    total = int(np.prod(sizes))
    out = np.zeros((total, total))
    for mu in range(d):
        # slots from slowest (x_d) to fastest (x_1)
        term = np.eye(1)
        for nu in reversed(range(d)):
            term = np.kron(term, mats[mu] if nu == mu else np.eye(sizes[nu]))
        out += term
    return out


def augmented_phi1(Kfull: np.ndarray, v: np.ndarray, tau: float) -> np.ndarray:
    """phi1(tau K) v as the top-right block of expm([[tau K, v], [0, 0]])."""
    from scipy.linalg import expm
    N = Kfull.shape[0]
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = tau * Kfull
    B[:N, N] = v
    return expm(B)[:N, N]
