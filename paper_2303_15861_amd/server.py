"""Python side of the request server (solve_submit / solve_poll of include/mumode.h).

Inputs are host numpy arrays; the server copies them, runs the solve on the device
in its own thread and keeps the result until it is polled.
"""
from __future__ import annotations

import sys
from ctypes import byref, c_uint64, c_void_p
from typing import Optional, Tuple

import numpy as np

# the package module itself (partly initialised while it imports this file), read at
# finalisation time without an import
_PKG = sys.modules[__package__]


class Server:
    def __init__(self, device: int = 0, max_active: int = 16, hbm_budget: int = 0):
        from . import _OPEN, MM_OK, MumodeError, lib
        self._lib = lib()
        self._h = c_void_p()
        self._shapes = {}          # request id -> shape of its solution
        st = self._lib.mm_server_create(device, max_active, int(hbm_budget), byref(self._h))
        if st != MM_OK:
            raise MumodeError(st, "mm_server_create failed")
        _OPEN.add(self)

    def clock(self) -> float:
        return self._lib.mm_server_clock(self._h)

    def counters(self) -> dict:
        """Launch counts of the step thread (mm_server_read_counters)."""
        from . import MM_OK, MMServerCounters, MumodeError
        c = MMServerCounters()
        st = self._lib.mm_server_read_counters(self._h, byref(c))
        if st != MM_OK:
            raise MumodeError(st, "mm_server_read_counters failed")
        out = {f: getattr(c, f) for f, _ in c._fields_}
        out["mean_group"] = c.problem_steps / c.group_steps if c.group_steps else 0.0
        return out

    def close(self):
        from . import _OPEN
        if self._h:
            self._lib.mm_server_destroy(self._h)
            self._h = c_void_p()
        _OPEN.discard(self)

    def __del__(self):
        if getattr(_PKG, "_EXITING", True):
            return
        try:
            self.close()
        except Exception:
            pass


def solve_submit(srv: Server, prob, prec: str = "fp64") -> Tuple[int, int]:
    """Queue a Lawson2b solve of a ``synth.Problem``; returns (status, id). The library
    copies (n+2)^d coefficient values (d fields of dof values for periodic problems) and
    dof initial values from the arrays, so their sizes are checked here first."""
    from . import FORMS, MM_BC_PERIODIC, MM_OK, MMRequest, coefficient_size, prec_code
    req = MMRequest()
    req.d = prob.d
    a = np.ascontiguousarray(prob.a, dtype=np.float64)
    u0 = np.ascontiguousarray(prob.u0, dtype=np.float64)
    periodic = bool(getattr(prob, "bc", ())) and prob.bc[0] == MM_BC_PERIODIC
    dof = int(np.prod([int(prob.n[i]) for i in range(prob.d)]))
    if a.size != coefficient_size(prob.d, prob.n, periodic):
        raise ValueError(f"a has {a.size} values, the request needs {coefficient_size(prob.d, prob.n, periodic)}")
    if u0.size != dof:
        raise ValueError(f"u0 has {u0.size} values, the request needs {dof}")
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
        if not periodic or vel.size != prob.d * dof:
            raise ValueError("a velocity field needs a periodic request and d * dof values")
        req.velocity = vel.ctypes.data   # copied by solve_submit before it returns
    rid = c_uint64()
    st = srv._lib.solve_submit(srv._h, byref(req), byref(rid))
    if st == MM_OK:
        srv._shapes[rid.value] = tuple(int(prob.n[i]) for i in reversed(range(prob.d)))
    return st, rid.value


def solve_poll(srv: Server, rid: int, shape=None) -> Tuple[int, Optional[np.ndarray], Optional[dict]]:
    """(status, solution or None, stats or None); status MM_NOT_READY while running. The
    solution buffer is sized from the request as submitted (the library copies the
    request's whole grid into it); `shape`, if given, must agree with it."""
    from . import MM_NOT_READY, MMStats
    own = srv._shapes.get(rid)
    if own is not None and shape is not None and int(np.prod(shape)) != int(np.prod(own)):
        raise ValueError(f"shape {tuple(shape)} does not match request {rid} of shape {own}")
    # an id not submitted through this wrapper gets no buffer (the library then copies
    # nothing): its size is not known here
    out = np.empty(own, dtype=np.float64) if own is not None else None
    stats = MMStats()
    st = srv._lib.solve_poll(srv._h, c_uint64(rid), out.ctypes.data if out is not None else None,
                             byref(stats))
    if st == MM_NOT_READY:
        return st, None, None
    srv._shapes.pop(rid, None)
    info = {"t_submit": stats.t_submit, "t_admit": stats.t_admit, "t_done": stats.t_done,
            "bytes": stats.bytes, "steps": stats.steps, "status": stats.status}
    return st, (out if st == 0 else None), info
