"""Python binding of the mu-mode exponential-integrator library (libmumode.so, gfx950).

Argument marshalling only: every step of the path runs in the HIP kernels of the
shared library behind the C ABI declared in include/mumode.h. PyTorch is used for
device memory (tensors) and streams; nothing here computes on grid data, and there
is no CPU fallback -- importing the binding raises if the library is missing.

Names follow the C ABI: mumode_setup, remainder_eval, mumode_expv, mumode_phi1v,
lawson_step, erk_step, mm_check, solve_submit, solve_poll.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from ctypes import POINTER, Structure, byref, c_char_p, c_double, c_int, c_int64, c_uint64, c_void_p
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmumode.so")

MM_OK, MM_NOT_READY = 0, 1
MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_EUNSTABLE, MM_EBUSY, MM_ENOTFOUND = -1, -2, -3, -4, -5, -6
MM_FP64, MM_FP32, MM_BF16X3, MM_BF16X6 = 0, 1, 2, 3
MM_LAWSON, MM_ERK = 0, 1
MM_LAWSON_EULER, MM_LAWSON2B = 0, 1
MM_ETD2RK, MM_ERK2P1 = 0, 1

MM_SLICED = 4
PRECISIONS = {"fp64": MM_FP64, "fp32": MM_FP32, "bf16x3": MM_BF16X3, "bf16x6": MM_BF16X6}
# exact slicing with S balanced base-256 digits: "sliced3" .. "sliced7"
PRECISIONS.update({f"sliced{s}": MM_SLICED for s in range(3, 8)})


def prec_code(prec: str):
    """(mm_prec, slices) of a precision name."""
    if prec not in PRECISIONS:
        raise ValueError(f"unknown precision {prec!r}; one of {sorted(PRECISIONS)}")
    return PRECISIONS[prec], (int(prec[6:]) if prec.startswith("sliced") else 0)
SCHEMES = {"le": (MM_LAWSON, MM_LAWSON_EULER), "l2b": (MM_LAWSON, MM_LAWSON2B),
           "sle": (MM_LAWSON, 2), "l2a": (MM_LAWSON, 3), "sl2": (MM_LAWSON, 4),
           "etd2rk": (MM_ERK, MM_ETD2RK), "erk2p1f": (MM_ERK, MM_ERK2P1),
           # exact phi functions only (q = 0)
           "ee": (MM_ERK, 2), "erk2p2": (MM_ERK, 3)}
STATUS = {0: "MM_OK", 1: "MM_NOT_READY", -1: "MM_EINVAL", -2: "MM_ENOMEM", -3: "MM_EDEVICE",
          -4: "MM_EUNSTABLE", -5: "MM_EBUSY", -6: "MM_ENOTFOUND"}

# every entry point the header declares
EXPORTS = ("mm_ctx_create", "mm_ctx_destroy", "mm_last_error", "mm_version", "mumode_setup",
           "mumode_destroy", "mumode_info", "mumode_get_factor", "remainder_eval", "mumode_expv",
           "mumode_phi1v", "lawson_step", "erk_step", "mm_check", "mm_server_create",
           "mm_server_destroy", "solve_submit", "solve_poll", "mm_server_clock", "mm_timing_enable",
           "mm_timing_read", "mm_synchronize", "mm_set_gemm_tile",
           "mm_set_graph_steps", "mm_set_small_fused", "lawson_step_batch",
           "mm_server_read_counters", "mumode_expv_noalloc", "mm_set_sliced_chain",
           "mm_set_fold")
MM_KIND_STENCIL, MM_KIND_GEMM_K, MM_KIND_GEMM_N, MM_KIND_FUSED = 0, 1, 2, 3


class MMProblem(Structure):
    _fields_ = [("d", c_int), ("n", c_int * 3), ("a", c_void_p), ("beta", c_double * 3),
                ("r", c_double * 4), ("lam", c_double), ("beta_bar", c_double * 3), ("bc", c_int * 3),
                ("form", c_int), ("length", c_double * 3), ("velocity", c_void_p)]


# boundary data per axis and diffusion form (mumode.h)
MM_BC_DIRICHLET, MM_BC_NEUMANN, MM_BC_PERIODIC = 0, 1, 2
MM_FORM_FLUX, MM_FORM_NONDIV = 0, 1
FORMS = {"flux": MM_FORM_FLUX, "nondiv": MM_FORM_NONDIV}


class MMRequest(Structure):
    _fields_ = [("d", c_int), ("n", c_int * 3), ("a", c_void_p), ("u0", c_void_p),
                ("beta", c_double * 3), ("r", c_double * 4), ("lam", c_double),
                ("beta_bar", c_double * 3), ("tau", c_double), ("steps", c_int), ("prec", c_int),
                ("slices", c_int), ("bc", c_int * 3), ("form", c_int), ("length", c_double * 3),
                ("velocity", c_void_p)]


class MMStats(Structure):
    _fields_ = [("t_submit", c_double), ("t_admit", c_double), ("t_done", c_double),
                ("bytes", c_int64), ("steps", c_int), ("status", c_int)]


class MMServerCounters(Structure):
    _fields_ = [("ticks", c_int64), ("group_launches", c_int64), ("group_steps", c_int64),
                ("problem_steps", c_int64), ("small_launches", c_int64), ("small_solves", c_int64),
                ("single_solves", c_int64)]


class MumodeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _hip_runtimes() -> set:
    """Files of HIP runtimes mapped into this process (Linux)."""
    try:
        with open("/proc/self/maps") as f:
            return {l.split()[-1] for l in f if "libamdhip64" in l}
    except OSError:
        return set()


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmumode.so and declare its signatures. Raises if it is not built.

    torch is imported first: its own HIP runtime (a libamdhip64 with the same SONAME as
    the one libmumode.so is linked against) is then already mapped, so the dynamic
    loader resolves libmumode's dependency to it and the process holds one runtime.
    Loaded the other way round, the process would map two runtimes, each with its own
    view of the device, and torch would report that no GPU is available."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2303_15861_amd.build "
                          "(there is no CPU fallback)")
    import torch  # noqa: F401  (maps torch's HIP runtime before libmumode.so)
    lib = ctypes.CDLL(path)
    if len(_hip_runtimes()) > 1:
        raise ImportError(f"two HIP runtimes are mapped ({sorted(_hip_runtimes())}); "
                          "libmumode.so must share torch's runtime")
    vp, i, d = c_void_p, c_int, c_double
    sig = {
        "mm_ctx_create": (i, [i, POINTER(vp)]),
        "mm_ctx_destroy": (None, [vp]),
        "mm_last_error": (c_char_p, [vp]),
        "mm_version": (c_char_p, []),
        "mumode_setup": (i, [vp, POINTER(MMProblem), d, i, i, i, i, i, POINTER(vp)]),
        "mumode_destroy": (None, [vp]),
        "mumode_info": (i, [vp, POINTER(c_double), POINTER(c_int)]),
        "mumode_get_factor": (i, [vp, i, i, vp]),
        "remainder_eval": (i, [vp, vp, vp, vp, vp, vp]),
        "mumode_expv": (i, [vp, vp, i, vp, vp, vp]),
        "mumode_phi1v": (i, [vp, vp, vp, vp, vp]),
        "mumode_expv_noalloc": (i, [vp, i, POINTER(c_int), POINTER(vp), vp, vp, vp]),
        "lawson_step": (i, [vp, vp, vp, i, vp]),
        "erk_step": (i, [vp, vp, vp, i, vp]),
        "lawson_step_batch": (i, [vp, POINTER(vp), POINTER(vp), i, i, vp]),
        "mm_check": (i, [vp, vp, vp]),
        "mm_server_create": (i, [i, i, c_int64, POINTER(vp)]),
        "mm_server_destroy": (None, [vp]),
        "solve_submit": (i, [vp, POINTER(MMRequest), POINTER(c_uint64)]),
        "solve_poll": (i, [vp, c_uint64, vp, POINTER(MMStats)]),
        "mm_server_clock": (d, [vp]),
        "mm_server_read_counters": (i, [vp, POINTER(MMServerCounters)]),
        "mm_timing_enable": (i, [vp, i]),
        "mm_synchronize": (i, [vp]),
        "mm_set_gemm_tile": (i, [vp, i]),
        "mm_set_graph_steps": (i, [vp, i]),
        "mm_set_small_fused": (i, [vp, i]),
        "mm_set_sliced_chain": (i, [vp, i]),
        "mm_set_fold": (i, [vp, i]),
        "mm_timing_read": (i, [vp, i, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _torch():
    import torch
    return torch


def _ptr(t, numel: Optional[int] = None, what: str = "grid tensor", device: Optional[int] = None) -> int:
    """Device address of a contiguous float64 GPU tensor of exactly `numel` values (when
    given) on `device` (when given). The kernels index the buffers by the problem's sizes
    alone, so a shorter tensor would be read or written past its end."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: has {t.numel()} values, the problem needs {numel}")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what}: must be a contiguous float64 tensor on the GPU")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: is on cuda:{t.device.index}, the context on cuda:{device}")
    return t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def coefficient_size(d: int, n: Sequence[int], periodic: bool) -> int:
    """Values of the diffusion coefficient a: the padded nodes (n_mu + 2 per axis), or for
    periodic problems the d diagonal fields on the grid."""
    dof, nodes = 1, 1
    for i in range(d):
        dof *= int(n[i])
        nodes *= int(n[i]) + 2
    return d * dof if periodic else nodes


# Library objects still open, released in order (servers, then operators through their
# contexts) by the exit handler below while the HIP runtime is certainly alive; once it
# has run, finalisers do nothing. Without it, objects that outlive the test or script
# (held by a traceback, a module global or a reference cycle) are released from the
# garbage collector during interpreter shutdown, in no particular order.
_OPEN = weakref.WeakSet()
_EXITING = False


@atexit.register
def _release_all():
    global _EXITING
    live = list(_OPEN)
    for obj in live:
        if isinstance(obj, Server):
            obj.close()
    for obj in live:
        if isinstance(obj, Context):
            obj.close()
    _EXITING = True


class Context:
    """An mm_ctx on one device."""

    def __init__(self, device: int = 0):
        self._h = c_void_p()
        self.device = device
        self._ops = weakref.WeakSet()     # live operators: released before the context
        st = lib().mm_ctx_create(device, byref(self._h))
        if st != MM_OK:
            raise MumodeError(st, f"mm_ctx_create(device={device}) failed")
        _OPEN.add(self)

    @property
    def handle(self):
        return self._h

    def error(self) -> str:
        return lib().mm_last_error(self._h).decode()

    def check(self, st: int, what: str):
        if st != MM_OK:
            raise MumodeError(st, f"{what}: {self.error()}")

    def timing(self, enable: bool):
        self.check(lib().mm_timing_enable(self._h, int(enable)), "mm_timing_enable")

    def set_gemm_tile(self, tile: int):
        """0: automatic; 32 (FP64 only), 64 or 128: force that workgroup tile for mode products."""
        self.check(lib().mm_set_gemm_tile(self._h, int(tile)), "mm_set_gemm_tile")

    def set_small_fused(self, enable: bool):
        """Whole small 2D Lawson solves in one workgroup (default on)."""
        self.check(lib().mm_set_small_fused(self._h, int(enable)), "mm_set_small_fused")

    def set_sliced_chain(self, mode: int):
        """Chained exact-slice actions of Lawson steps: 0 off, 1 automatic (default; every
        axis longer than 128), 2 wherever possible, 3 as 2 with four-wave workgroups."""
        self.check(lib().mm_set_sliced_chain(self._h, int(mode)), "mm_set_sliced_chain")

    def set_fold(self, mode: int):
        """FP64 folded mode products on centrosymmetric axes: 0 off, 1 on for products of at
        least 192 folded tiles per problem (default), 2 always."""
        self.check(lib().mm_set_fold(self._h, int(mode)), "mm_set_fold")

    def set_graph_steps(self, steps: int):
        """0: launch step kernels one by one; G > 0: replay recorded graphs of G steps."""
        self.check(lib().mm_set_graph_steps(self._h, int(steps)), "mm_set_graph_steps")

    def timing_read(self, kind: int):
        """(launches, total milliseconds, algorithmic work) of one kernel kind."""
        n, ms, wk = c_int64(), c_double(), c_double()
        self.check(lib().mm_timing_read(self._h, kind, byref(n), byref(ms), byref(wk)), "mm_timing_read")
        return n.value, ms.value, wk.value

    def close(self):
        if self._h:
            for op in list(self._ops):
                op.close()
            lib().mm_ctx_destroy(self._h)
            self._h = c_void_p()
        _OPEN.discard(self)

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """An mm_op: factors and scratch for one problem, time step and scheme."""

    def __init__(self, ctx: Context, handle: c_void_p, prob, scheme: str, prec: str, q: int):
        self.ctx, self._h = ctx, handle
        ctx._ops.add(self)
        self.d, self.n = prob.d, tuple(prob.n)
        self.scheme, self.prec, self.q = scheme, prec, q
        self.family = SCHEMES[scheme][0]
        self.dof = 1
        for i in range(self.d):
            self.dof *= self.n[i]

    @property
    def handle(self):
        return self._h

    @property
    def shape(self):
        return tuple(reversed(self.n[: self.d]))

    def grid(self, t, what: str = "grid tensor") -> int:
        """Address of a grid function of this operator's problem (checked size and device)."""
        if not self._h:
            raise ValueError("the operator is closed")
        return _ptr(t, self.dof, what, self.ctx.device)

    def info(self):
        am = c_double()
        sq = (c_int * 3)()
        lib().mumode_info(self._h, byref(am), sq)
        return am.value, tuple(sq[: self.d])

    def factor(self, mu: int, j: int = 0):
        import numpy as np
        n = self.n[mu]
        out = np.empty((n, n), dtype=np.float64)
        st = lib().mumode_get_factor(self._h, mu, j, out.ctypes.data)
        self.ctx.check(st, "mumode_get_factor")
        return out

    def close(self):
        # a closed context has released its operators first (Context.close), so an op
        # whose context is gone has nothing left to free
        if self._h and self.ctx.handle:
            # through the library, so that this is safe from a finaliser
            lib().mm_synchronize(self.ctx.handle)
            lib().mumode_destroy(self._h)
        self._h = c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


def mumode_setup(ctx: Context, d: int, n: Sequence[int], a, beta: Sequence[float], r: Sequence[float],
                 tau: float, scheme: str = "l2b", prec: str = "fp64", q: int = 4, lam: float = 1.0,
                 beta_bar: Optional[Sequence[float]] = None, bc: Optional[Sequence[int]] = None,
                 form: str = "flux", length: Optional[Sequence[float]] = None, velocity=None) -> Operator:
    """Build the extracted operator and its factors on the device (see mumode.h). For
    periodic problems ``a`` holds the d diagonal diffusion fields and ``velocity`` (a
    device tensor or None) the d velocity fields; ``length`` gives the periods."""
    prob = MMProblem()
    prob.d = d
    for i in range(3):
        prob.n[i] = int(n[i]) if i < d else 1
        prob.beta[i] = float(beta[i]) if i < d else 0.0
        prob.beta_bar[i] = float(beta_bar[i]) if (beta_bar is not None and i < d) else 0.0
        prob.bc[i] = int(bc[i]) if (bc is not None and i < d) else MM_BC_DIRICHLET
    prob.form = FORMS[form]
    for i in range(4):
        prob.r[i] = float(r[i])
    prob.lam = float(lam)
    periodic = prob.bc[0] == MM_BC_PERIODIC
    # sizes are checked for a well-formed problem; the library refuses any other (MM_EINVAL)
    # before it reads a buffer
    sized = d in (2, 3) and all(prob.n[i] >= 1 for i in range(d))
    dof = 1
    for i in range(min(d, 3)):
        dof *= prob.n[i]
    prob.a = _ptr(a, coefficient_size(d, prob.n, periodic) if sized else None, "diffusion coefficient a",
                  ctx.device)
    for i in range(3):
        prob.length[i] = float(length[i]) if (length is not None and i < d) else 0.0
    prob.velocity = (_ptr(velocity, d * dof if sized else None, "velocity", ctx.device)
                     if velocity is not None else None)
    _torch().cuda.current_stream(a.device).synchronize()   # a must be complete
    fam, sch = SCHEMES[scheme]
    h = c_void_p()
    code, slices = prec_code(prec)
    st = lib().mumode_setup(ctx.handle, byref(prob), float(tau), fam, sch, int(q), code, slices,
                            byref(h))
    ctx.check(st, "mumode_setup")
    return Operator(ctx, h, prob, scheme, prec, q if fam == MM_ERK else 0)


def remainder_eval(op: Operator, u, g, F=None, stream=None):
    st = lib().remainder_eval(op.ctx.handle, op.handle, op.grid(u, "u"), op.grid(g, "g"),
                              op.grid(F, "F") if F is not None else None, _stream(stream))
    op.ctx.check(st, "remainder_eval")


def mumode_expv(op: Operator, inp, out, j: int = 0, stream=None):
    st = lib().mumode_expv(op.ctx.handle, op.handle, int(j), op.grid(inp, "input"), op.grid(out, "output"),
                           _stream(stream))
    op.ctx.check(st, "mumode_expv")


def mumode_phi1v(op: Operator, inp, out, stream=None):
    st = lib().mumode_phi1v(op.ctx.handle, op.handle, op.grid(inp, "input"), op.grid(out, "output"),
                            _stream(stream))
    op.ctx.check(st, "mumode_phi1v")


def lawson_step(op: Operator, u, nsteps: int, stream=None):
    st = lib().lawson_step(op.ctx.handle, op.handle, op.grid(u, "u"), int(nsteps), _stream(stream))
    op.ctx.check(st, "lawson_step")


NOALLOC_MAX_DOF = 1 << 21


def mumode_expv_noalloc(ctx: Context, factors, inp, out, stream=None):
    """out = inp x_mu factors[mu] over the axes (FP64), with no device allocation: the
    intermediates use the library's per-device scratch array (see mumode.h)."""
    d = len(factors)
    n = [int(f.shape[0]) for f in factors]
    for f in factors:
        if f.dim() != 2 or f.shape[0] != f.shape[1]:
            raise ValueError("every factor must be a square matrix")
    dof = 1
    for m in n:
        dof *= m
    hn = (c_int * 3)(*(n + [1] * (3 - d)))
    hE = (c_void_p * d)(*[_ptr(f, f.shape[0] * f.shape[1], f"factor {mu}", ctx.device) for mu, f in enumerate(factors)])
    st = lib().mumode_expv_noalloc(ctx.handle, d, hn, hE, _ptr(inp, dof, "input", ctx.device),
                                   _ptr(out, dof, "output", ctx.device), _stream(stream))
    ctx.check(st, "mumode_expv_noalloc")


def lawson_step_batch(ops: Sequence[Operator], us, nsteps: int, stream=None):
    """Grouped Lawson steps: ops[i] advances us[i] (one class: shape, precision, scheme)."""
    count = len(ops)
    if count != len(us) or count < 1:
        raise ValueError("lawson_step_batch needs as many states as operators (at least one)")
    ctx = ops[0].ctx
    if any(op.ctx is not ctx for op in ops):
        raise ValueError("lawson_step_batch: every operator must come from the same context")
    hops = (c_void_p * count)(*[op.handle.value for op in ops])
    hus = (c_void_p * count)(*[op.grid(u, f"u[{i}]") for i, (op, u) in enumerate(zip(ops, us))])
    st = lib().lawson_step_batch(ctx.handle, hops, hus, count, int(nsteps), _stream(stream))
    ctx.check(st, "lawson_step_batch")


def erk_step(op: Operator, u, nsteps: int, stream=None):
    st = lib().erk_step(op.ctx.handle, op.handle, op.grid(u, "u"), int(nsteps), _stream(stream))
    op.ctx.check(st, "erk_step")


def step(op: Operator, u, nsteps: int, stream=None):
    """lawson_step or erk_step according to the operator's family."""
    if op.family == MM_LAWSON:
        lawson_step(op, u, nsteps, stream)
    else:
        erk_step(op, u, nsteps, stream)


def mm_check(op: Operator, stream=None) -> int:
    """Synchronise the stream; returns MM_OK or MM_EUNSTABLE (raises on other errors)."""
    st = lib().mm_check(op.ctx.handle, op.handle, _stream(stream))
    if st not in (MM_OK, MM_EUNSTABLE):
        op.ctx.check(st, "mm_check")
    return st


def setup_problem(ctx: Context, prob, prec: str = "fp64", scheme: Optional[str] = None) -> Operator:
    """mumode_setup for a ``synth.Problem`` (copies its coefficient to the device)."""
    torch = _torch()
    import numpy as np
    dev = f"cuda:{ctx.device}"
    a = torch.from_numpy(np.ascontiguousarray(prob.a)).to(device=dev)
    vel = getattr(prob, "velocity", None)
    vel = torch.from_numpy(np.ascontiguousarray(vel)).to(device=dev) if vel is not None else None
    op = mumode_setup(ctx, prob.d, prob.n, a, prob.beta, prob.r, prob.tau, scheme or prob.scheme, prec,
                      prob.q, prob.lam, prob.beta_bar, getattr(prob, "bc", None), getattr(prob, "form", "flux"),
                      getattr(prob, "length", None) or None, vel)
    return op


from .server import Server, solve_poll, solve_submit  # noqa: E402,F401
