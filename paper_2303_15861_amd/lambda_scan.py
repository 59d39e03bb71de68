"""Choice of the extraction factor lambda by a scan on a coarse problem (end of Sec. 3).

The paper picks lambda in A = lambda a_max Lap + ... by running the scheme on a problem
with few degrees of freedom for each admissible lambda (from the scheme's stability
bound up to 1) and keeping the lambda with the smallest error against a reference
solution (Lawson2b with a small step, Sec. 5); the large solve then uses that lambda.
Every run here is a GPU solve through the C ABI.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np

# lower ends of the unconditionally stable lambda range for each scheme as printed in
# Table tab:stab (stabilized Lawson2 with alpha = 0.327; the ERK2 with phi1, c2 = 1, in
# either form)
STABILITY_BOUND = {"ee": 0.5, "erk2p2": 0.5, "erk2p1f": 1.0 / 3.0, "etd2rk": 1.0 / 3.0, "l2a": 0.301,
                   "l2b": 0.301, "le": 0.218, "sle": 0.5 / np.e, "sl2": 0.183}


def _solve(mm, ctx, prob, prec: str) -> np.ndarray:
    import torch
    op = mm.setup_problem(ctx, prob, prec=prec)
    try:
        u = torch.from_numpy(np.ascontiguousarray(prob.u0)).to(f"cuda:{ctx.device}")
        mm.step(op, u, prob.steps)
        if mm.mm_check(op) != mm.MM_OK:
            return np.full(prob.shape, np.nan)
        torch.cuda.synchronize()
        return u.cpu().numpy()
    finally:
        op.close()


def lambda_scan(ctx, coarse, lams: Optional[Sequence[float]] = None, *, points: int = 20,
                ref_steps: int = 2 ** 14, prec: str = "fp64",
                reference: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray, float]:
    """Scan lambda for ``coarse`` (a synth.Problem: its scheme, step count and final time
    are kept, only lam changes). lams defaults to ``points`` values from the scheme's
    stability bound to 1. The reference is Lawson2b at lambda = 1 with ``ref_steps``
    steps to the same final time (or the given array). Returns (lams, relative
    infinity-norm errors at the final time, the lambda of the smallest error)."""
    import paper_2303_15861_amd as mm
    if lams is None:
        lams = np.linspace(STABILITY_BOUND[coarse.scheme], 1.0, points)
    lams = np.asarray(lams, dtype=float)
    if reference is None:
        T = coarse.tau * coarse.steps
        ref = dataclasses.replace(coarse, scheme="l2b", lam=1.0, steps=ref_steps, tau=T / ref_steps)
        reference = _solve(mm, ctx, ref, "fp64")
    scale = float(np.max(np.abs(reference)))
    errs = np.empty(len(lams))
    for i, lam in enumerate(lams):
        u = _solve(mm, ctx, dataclasses.replace(coarse, lam=float(lam)), prec)
        errs[i] = np.max(np.abs(u - reference)) / scale if np.all(np.isfinite(u)) else np.inf
    return lams, errs, float(lams[int(np.argmin(errs))])
