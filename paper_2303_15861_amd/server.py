"""Python side of the request server (solve_submit / solve_poll of include/mumode.h).

Inputs are host numpy arrays; the server copies them, runs the solve on the device
in its own thread and keeps the result until it is polled.
"""
from __future__ import annotations

from ctypes import byref, c_uint64, c_void_p
from typing import Optional, Tuple

import numpy as np


class Server:
    def __init__(self, device: int = 0, max_active: int = 16, hbm_budget: int = 0):
        from . import MM_OK, MumodeError, lib
        self._lib = lib()
        self._h = c_void_p()
        st = self._lib.mm_server_create(device, max_active, int(hbm_budget), byref(self._h))
        if st != MM_OK:
            raise MumodeError(st, "mm_server_create failed")

    def clock(self) -> float:
        return self._lib.mm_server_clock(self._h)

    def close(self):
        if self._h:
            self._lib.mm_server_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_submit(srv: Server, prob, prec: str = "fp64") -> Tuple[int, int]:
    """Queue a Lawson2b solve of a ``synth.Problem``; returns (status, id)."""
    from . import FORMS, MMRequest, prec_code
    req = MMRequest()
    req.d = prob.d
    a = np.ascontiguousarray(prob.a, dtype=np.float64)
    u0 = np.ascontiguousarray(prob.u0, dtype=np.float64)
    for i in range(3):
        req.n[i] = int(prob.n[i]) if i < prob.d else 1
        req.beta[i] = float(prob.beta[i]) if i < prob.d else 0.0
        req.beta_bar[i] = float(prob.beta_bar[i]) if i < prob.d else 0.0
        req.bc[i] = int(prob.bc[i]) if (i < prob.d and getattr(prob, "bc", ())) else 0
    req.form = FORMS[getattr(prob, "form", "flux")]
    for i in range(4):
        req.r[i] = float(prob.r[i])
    req.lam = float(prob.lam)
    req.tau = float(prob.tau)
    req.steps = int(prob.steps)
    req.prec, req.slices = prec_code(prec)
    req.a = a.ctypes.data
    req.u0 = u0.ctypes.data
    length = getattr(prob, "length", ()) or ()
    for i in range(3):
        req.length[i] = float(length[i]) if i < len(length) else 0.0
    vel = getattr(prob, "velocity", None)
    if vel is not None:
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        req.velocity = vel.ctypes.data   # copied by solve_submit before it returns
    rid = c_uint64()
    st = srv._lib.solve_submit(srv._h, byref(req), byref(rid))
    return st, rid.value


def solve_poll(srv: Server, rid: int, shape) -> Tuple[int, Optional[np.ndarray], Optional[dict]]:
    """(status, solution or None, stats or None); status MM_NOT_READY while running."""
    from . import MM_NOT_READY, MMStats
    out = np.empty(shape, dtype=np.float64)
    stats = MMStats()
    st = srv._lib.solve_poll(srv._h, c_uint64(rid), out.ctypes.data, byref(stats))
    if st == MM_NOT_READY:
        return st, None, None
    info = {"t_submit": stats.t_submit, "t_admit": stats.t_admit, "t_done": stats.t_done,
            "bytes": stats.bytes, "steps": stats.steps, "status": stats.status}
    return st, (out if st == 0 else None), info
