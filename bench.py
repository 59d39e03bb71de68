"""Benchmark: Mdof*steps/s of the mu-mode Lawson2b path on the 255^3 workload.

One step = one Lawson2b step over the whole grid: two fused remainder/stage passes and
one stacked exp action (three mode products on two grid functions). The workload is the
3D Dirichlet ADR problem with 255^3 interior points (h = 1/256), a = 1 + 0.9 tanh(s),
beta = (10, 10, 10), r = u^2(1 - u), tau = 1e-3, 100 steps to T = 0.1 (synthetic seeded
inputs). Every contraction precision is timed; the headline value is the FP64 path
unless --headline names another mode. Each mode is also run untimed over the whole
interval to T and its error stated there: against the FP64 path on the whole grid and
against the CPU oracle on its stored samples (tests/golden/oracle_3d_n255_l2b_T.txt),
with the stated target of the mode (FP32 1e-6, split modes 1e-9) as pass/fail.

The served stream (512 seeded requests at 200/s) runs in FP64 with step-level batching,
in FP64 one request at a time (max_active = 1), and in the sliced mode that meets the
split target. The other workloads (63^2 Lawson-Euler, 127^3 Lawson2b and ETD2RK, 383^3
ETD2RK) get a line each under "configs" with their dominant kernel's roofline, and the
oracle is timed on bounded samples of each on the host ("cpu_baselines").

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes fp64,fp32,...]

Prints one JSON line. --gpus N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "int8": 5.0e15}
HBM_PEAK = 8.0e12
DESCRIPTION = {
    "3d_n255_l2b": "3D Dirichlet ADR 255^3 interior, Lawson2b, tau=1e-3, 100 steps to T=0.1",
    "3d_n127_l2b": "3D Dirichlet ADR 127^3 interior, Lawson2b, tau=5e-4, 200 steps to T=0.1",
    "3d_n127_etd2rk": "3D Dirichlet ADR 127^3 interior, ETD2RK with 4-node phi1, tau=5e-4, 200 steps",
    "3d_n383_etd2rk": "3D Dirichlet ADR 383^3 interior, anisotropic a in (0.01, 2), ETD2RK with 6-node "
                      "phi1, tau=2e-3, 50 steps",
    "2d_n63_le": "2D Dirichlet ADR 63^2 interior, Lawson-Euler, tau=1e-3, 100 steps",
    "3d_n127_etd2rk_exact": "3D Dirichlet ADR 127^3 interior, ETD2RK with exact phi1 (eigenbasis), tau=5e-4, "
                            "200 steps",
    "3d_n383_etd2rk_exact": "3D Dirichlet ADR 383^3 interior, anisotropic a in (0.01, 2), ETD2RK with exact "
                            "phi1 (eigenbasis), tau=2e-3, 50 steps",
    "3d_paper_n60_sl2": "the 3D ADR problem of Sec. 5.2 (a Lap u, Dirichlet at 0, Neumann at 1), N = 60, b = -0.01, "
                        "SL2 with lambda = 0.53, 256 steps to T = 1/4",
    "2d_paper_n256_sl2": "the periodic 2D ADR problem of Sec. 5.1 (pseudo-spectral, circulant factors), N = 256, "
                         "SL2 with lambda = 0.57, 256 steps to T = 4",
}
WORKLOAD = "3d_n255_l2b"
# stated error targets of the contraction modes at T (FP32; split / sliced modes)
TARGET = {"fp32": 1e-6, "bf16x3": 1e-9, "bf16x6": 1e-9}
# other workloads: (name, timed steps or None for the whole solve, precisions)
CONFIGS = [("2d_n63_le", None, ("fp64",)), ("3d_n127_l2b", None, ("fp64", "sliced5")),
           ("3d_n127_etd2rk", None, ("fp64",)), ("3d_n383_etd2rk", 5, ("fp64", "sliced5"))]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default=WORKLOAD, help="one of synth.WORKLOADS")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--modes", default="fp64,fp32,bf16x6,bf16x3,sliced4,sliced5,sliced6,sliced7")
    ap.add_argument("--headline", default="fp64")
    ap.add_argument("--latency-reps", type=int, default=20)
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="replay step loops from recorded HIP graphs of this many steps (0: direct launches)")
    ap.add_argument("--tile", type=int, default=0, help="force the mode-product workgroup tile (64 or 128)")
    ap.add_argument("--sliced-chain", type=int, default=1,
                    help="chained exact-slice actions: 0 off, 1 automatic, 2 always, 3 four-wave workgroups")
    ap.add_argument("--fold", type=int, default=1,
                    help="FP64 folded mode products on centrosymmetric axes: 0 off, 1 automatic, 2 always")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-at-T", action="store_true", help="skip the untimed runs to T")
    ap.add_argument("--serve", default="fp64,sliced5",
                    help="precisions for the served-stream run ('' to skip)")
    ap.add_argument("--serve-count", type=int, default=512)
    ap.add_argument("--serve-active", type=int, default=32)
    ap.add_argument("--no-serial", action="store_true", help="skip the one-at-a-time served-stream baseline")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads")
    ap.add_argument("--calibrate", action="store_true",
                    help="run a plain elementwise copy of one grid function (known bytes) first, "
                         "as the reference for HBM counter runs")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_f64_255cube_l2b_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2303_15861_amd", "csrc", "contract.hip")


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m_sha = re.search(r"contract\.hip sha1: ([0-9a-f]{40})", text)
    m_bytes = re.search(r"traffic per launch \(bytes\): ([0-9.eE+]+)", text)
    if not m_sha or not m_bytes:
        return None
    sha = hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()
    return float(m_bytes.group(1)) if sha == m_sha.group(1) else None


def oracle_samples(workload):
    """(max |u(T)|, flat indices, values) of the oracle at T, or None without a fixture."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_T.txt")
    if not os.path.exists(path):
        return None
    idx, val, mx = [], [], None
    for line in open(path):
        if line.startswith("#"):
            continue
        a, b = line.split()
        if a == "max_abs":
            mx = float.fromhex(b)
        else:
            idx.append(int(a))
            val.append(float.fromhex(b))
    return mx, np.array(idx, dtype=np.int64), np.array(val)


def dtype_name(prec):
    """Arithmetic type of a mode's contractions."""
    if prec.startswith("sliced"):
        return f"i8x{prec[6:]}"          # S int8 digit planes, int32 accumulation, f64 combination
    return {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[prec]


def target(prec):
    if prec == "fp64":
        return None
    return 1e-9 if prec.startswith("sliced") else TARGET[prec]


def slice_products(prec):
    S = int(prec[6:])
    return S * (S + 1) // 2


# Untimed steps before each timed region run for at least this long: under sustained
# load the GPU's clocks take a few tenths of a second to settle (the 255^3 mode products
# go from about 390 to about 300 us per launch over the first 25 steps of a cold run), so
# a warmup of a few steps alone would time the ramp.
WARMUP_MIN_S = 0.5


def time_mode(mm, ctx, p, prec, steps, warmup, graph_steps=0):
    """Timed region: `steps` steps on a resident state, no per-kernel events. Before it,
    `warmup` untimed steps and then more until WARMUP_MIN_S of steps have run. A second,
    untimed pass of the same steps brackets every kernel with HIP events on its stream
    for the per-kernel table and the roofline. With graph replay the warmup runs at
    least one graph's worth of steps, so that the graph is recorded before timing."""
    import torch
    op = mm.setup_problem(ctx, p, prec=prec)
    u0 = torch.from_numpy(p.u0).to("cuda")
    u = u0.clone()
    stream = torch.cuda.current_stream()
    warmup = max(warmup, graph_steps)
    t0 = time.perf_counter()
    if warmup:
        mm.step(op, u, warmup, stream)
    torch.cuda.synchronize()
    chunk = max(1, warmup)
    while time.perf_counter() - t0 < WARMUP_MIN_S:
        u.copy_(u0)
        mm.step(op, u, chunk, stream)
        torch.cuda.synchronize()
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mm.step(op, u, steps, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    status = mm.mm_check(op)
    out = u.cpu().numpy()
    u.copy_(u0)
    torch.cuda.synchronize()
    ctx.timing(True)
    mm.step(op, u, steps, stream)
    kern = {}
    for kind, name in ((mm.MM_KIND_GEMM_K, "gemm_k"), (mm.MM_KIND_GEMM_N, "gemm_n"),
                       (mm.MM_KIND_STENCIL, "stencil"), (mm.MM_KIND_FUSED, "fused")):
        n, ms, wk = ctx.timing_read(kind)
        kern[name] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / max(n, 1), "work": wk}
    ctx.timing(False)
    return op, out, (t1 - t0), kern, status


def run_to_T(mm, op, p):
    """The whole solve (p.steps steps from u0), untimed; the state at T on the host."""
    import torch
    u = torch.from_numpy(p.u0).to("cuda")
    mm.step(op, u, p.steps)
    status = mm.mm_check(op)
    return u.cpu().numpy(), status


def roofline(kern, prec, p):
    """Roofline of the dominant kernel kind of one timed run (algorithmic work per launch
    over the launch durations measured with HIP events on the launch streams)."""
    kname = max(("gemm_k", "gemm_n", "stencil", "fused"), key=lambda k: kern[k]["total_ms"])
    k = kern[kname]
    secs = k["total_ms"] * 1e-3
    if kname == "fused":
        # one workgroup per solve on one compute unit: its share of the FP64 matrix peak
        roof = {"bound": "mfma", "achieved": k["work"] / secs / 1e12, "peak": PEAK["fp64"] / 256 / 1e12,
                "unit": "TFLOP/s", "scope": "one compute unit"}
    elif kname == "stencil":
        # algorithmic bytes per grid point of a fused remainder pass: read u and a, write
        # two outputs (first pass) or read U, W, a and write u (second pass): 32 B
        roof = {"bound": "hbm", "achieved": 32.0 * k["work"] / secs / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s"}
    elif prec.startswith("sliced"):
        # int8 digit products executed, S(S+1)/2 per algorithmic multiply-add. Chained
        # Lawson steps (every axis of 129..256 points under the default chain mode): each
        # product's epilogue writes the next mode's digits; otherwise the launch time also
        # includes the pass that splits the grid operand into digits
        chained = p.scheme in ("le", "l2b") and all(128 < m <= 256 for m in p.n)
        roof = {"bound": "mfma", "achieved": k["work"] * slice_products(prec) / secs / 1e12,
                "peak": PEAK["int8"] / 1e12, "unit": "TOP/s",
                "includes": ("chained int8 product (its epilogue writes the next mode's digit planes)" if chained
                             else "grid split + int8 product")}
    elif prec in ("bf16x3", "bf16x6"):
        # split-BF16 contractions are bound by HBM: 16 B per grid point per pass
        bytes_ = 16.0 * k["work"] / (2.0 * p.n[0])
        roof = {"bound": "hbm", "achieved": bytes_ / secs / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": k["work"] / secs / 1e12, "peak": PEAK[prec] / 1e12,
                "unit": "TFLOP/s"}
        if prec == "fp64" and p.scheme in ("le", "l2b") and kname in ("gemm_k", "gemm_n"):
            # folded products (centrosymmetric factors) execute about half the FP64 work of
            # the plain product 2 n_mu dof per vector; the library reports the executed work
            nmu = p.n[0] if kname == "gemm_k" else p.n[-1]
            plain = k["launches"] * 2.0 * nmu * float(np.prod(p.n)) * (2 if p.scheme == "l2b" else 1)
            if k["work"] < 0.75 * plain:
                roof["folded"] = True
                roof["plain_equivalent_tflops"] = plain / secs / 1e12
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = {"gemm_k": "gemm (mode 1)", "gemm_n": "gemm (modes 2, 3)", "stencil": "stencil",
                      "fused": "whole small-2D solve in one workgroup (one compute unit)"}[kname]
    roof["avg_launch_us"] = k["avg_us"]
    return roof, kname


def latency(mm, ctx, op, p, reps):
    import torch
    u0 = torch.from_numpy(p.u0).to("cuda")
    u = u0.clone()
    lat = []
    for _ in range(reps):
        u.copy_(u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mm.step(op, u, p.steps)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "reps": reps, "steps_per_solve": p.steps}


def serve_stream(mm, prec, count, max_active):
    """The served stream: `count` seeded Lawson2b solves (50% 2D N in {64..512}^2, 50% 3D
    N in {32..192}^3, beta ~ U[0,20]^d, f = u(1-u) or u^2(1-u), 20-200 steps to T = 0.1)
    submitted at Poisson arrival times (200/s). Latency = completion - submission on the
    server clock."""
    import synth
    reqs = synth.request_stream(count=count, seed=1)
    probs = [r.problem() for r in reqs]          # generated before the clock starts
    srv = mm.Server(0, max_active=max_active)
    ids = []
    t0 = time.perf_counter()
    for r, p in zip(reqs, probs):
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        st, rid = mm.solve_submit(srv, p, prec=prec)
        ids.append((rid, p))
    lat, done, statuses, work = [], [], {}, 0.0
    t_first = None
    pending = list(ids)
    while pending:
        rest = []
        for rid, p in pending:
            st, u, info = mm.solve_poll(srv, rid)
            if st == mm.MM_NOT_READY:
                rest.append((rid, p))
                continue
            statuses[mm.STATUS.get(st, st)] = statuses.get(mm.STATUS.get(st, st), 0) + 1
            if info:
                lat.append(info["t_done"] - info["t_submit"])
                done.append(info["t_done"])
                t_first = info["t_submit"] if t_first is None else min(t_first, info["t_submit"])
                work += p.dof * p.steps
        pending = rest
        if pending:
            time.sleep(0.002)
    counters = srv.counters()
    srv.close()
    lat = np.array(lat) * 1e3
    span = max(done) - t_first
    return {"requests": count, "max_active": max_active, "status": statuses,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": span,
            "throughput_mdof_steps_per_s": work / span / 1e6,
            "mean_requests_per_grouped_launch": counters["mean_group"],
            "launches": {k: v for k, v in counters.items() if k != "mean_group"}}


def oracle_module(p):
    import synth
    if any(b == synth.PERIODIC for b in getattr(p, "bc", ())):
        from oracle import spectral as S       # periodic pseudo-spectral problems
    elif any(getattr(p, "bc", ())) or getattr(p, "form", "flux") != "flux":
        from oracle import adr3d as S          # Neumann axes or the non-divergence form
    else:
        from oracle import schemes as S
    return S


def time_oracle(p, steps, threads):
    """Seconds of `steps` oracle steps of p with the BLAS pool limited to `threads`."""
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=threads)
    except Exception:  # pragma: no cover
        lim = None
    S = oracle_module(p)
    t0 = time.perf_counter()
    S.solve(p, steps=steps)
    dt = time.perf_counter() - t0
    if lim is not None and hasattr(lim, "unregister"):
        lim.unregister()
    return dt


def cpu_baseline(p, steps):
    """The oracle, untuned, on the host cores: `steps` steps of the workload's scheme."""
    cores = len(os.sched_getaffinity(0))
    dt = time_oracle(p, steps, cores)
    return {"value": p.dof * steps / dt / 1e6, "unit": "Mdof*steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} {p.scheme} steps of the {p.name} workload (numpy FP64, OpenBLAS threads = cores)",
            "seconds": dt}


def cpu_baselines():
    """The oracle on bounded samples of the other workloads (BLAS threads = cores, and one
    thread for the 63^2 solve), and on a seeded 64-request subset of the served stream."""
    import synth
    cores = len(os.sched_getaffinity(0))
    out = {}
    p = synth.workload("2d_n63_le")
    for th in (1, cores):
        dt = time_oracle(p, p.steps, th)
        out[f"2d_n63_le_threads{th}"] = {"us_per_step": 1e6 * dt / p.steps, "threads": th,
                                         "sample": f"whole solve, {p.steps} steps"}
    for name, steps in (("3d_n127_l2b", 4), ("3d_n127_etd2rk", 2), ("3d_n383_etd2rk", 1)):
        p = synth.workload(name)
        dt = time_oracle(p, steps, cores)
        out[name] = {"ms_per_step": 1e3 * dt / steps, "mdof_steps_per_s": p.dof * steps / dt / 1e6,
                     "threads": cores, "sample": f"{steps} steps"}
    # served stream: 64 requests spread over every (d, n) bucket, 2 steps each
    reqs = synth.request_stream(count=512, seed=1)
    buckets = {}
    for r in reqs:
        buckets.setdefault((r.d, r.n), []).append(r)
    subset = []
    while len(subset) < 64 and any(buckets.values()):
        for key in sorted(buckets):
            if buckets[key] and len(subset) < 64:
                subset.append(buckets[key].pop(0))
    t0 = time.perf_counter()
    dofsteps = 0
    for r in subset:
        q = r.problem()
        time_oracle(q, 2, cores)
        dofsteps += q.dof * 2
    dt = time.perf_counter() - t0
    out["served_stream_subset"] = {"mdof_steps_per_s": dofsteps / dt / 1e6, "requests": len(subset),
                                   "threads": cores, "seconds": dt,
                                   "sample": "64 requests of the 512-request stream, every (d, n) bucket, "
                                             "first 2 steps each"}
    return out


def config_lines(mm, ctx, warmup):
    """One line per other workload: ms/step, Mdof*steps/s and the dominant kernel's roofline;
    a mixed precision also states its error against the FP64 path after the same timed
    steps from the same initial state."""
    import synth
    out = {}
    for name, steps, precs in CONFIGS:
        p = synth.workload(name)
        nsteps = steps or p.steps
        ref = None
        for prec in precs:
            print(f"[bench] config {name} {prec}: {nsteps} timed steps", file=sys.stderr, flush=True)
            try:
                op, state, dt, kern, status = time_mode(mm, ctx, p, prec, nsteps, min(warmup, 2))
            except mm.MumodeError as exc:
                print(f"[bench] config {name} {prec}: {exc}", file=sys.stderr, flush=True)
                continue
            op.close()
            roof, _ = roofline(kern, prec, p)
            entry = {"workload": DESCRIPTION.get(name, name), "ms_per_step": 1e3 * dt / nsteps,
                     "value": p.dof * nsteps / dt / 1e6, "unit": "Mdof*steps/s",
                     "steps": nsteps, "status": mm.STATUS.get(status, status), "roofline": roof}
            if prec == "fp64":
                ref = state
            elif ref is not None:
                entry["err_vs_fp64_after_steps"] = float(np.max(np.abs(state - ref)) / np.max(np.abs(ref)))
            out[f"{name}_{prec}"] = entry
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2303_15861_amd as mm
    import synth

    p = synth.workload(args.workload)
    if args.calibrate:
        # plain copy kernel of known size: reads and writes dof doubles
        src = torch.from_numpy(p.u0).to("cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {p.dof * 8} bytes read and written per dispatch", file=sys.stderr,
              flush=True)
        del src, dst
    ctx = mm.Context(0)
    ctx.set_graph_steps(args.graph_steps)
    ctx.set_gemm_tile(args.tile)
    ctx.set_sliced_chain(args.sliced_chain)
    ctx.set_fold(args.fold)
    modes = [m for m in args.modes.split(",") if m]
    if "fp64" not in modes:
        modes = ["fp64"] + modes
    samples = oracle_samples(args.workload)
    res = {}
    ref, ref_T = None, None
    for prec in modes:
        print(f"[bench] {prec}: setup + {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
              flush=True)
        try:
            op, out, dt, kern, status = time_mode(mm, ctx, p, prec, args.steps, args.warmup, args.graph_steps)
        except mm.MumodeError as exc:
            if prec == "fp64":
                raise
            print(f"[bench] {prec}: not available for this workload ({exc})", file=sys.stderr, flush=True)
            continue
        entry = {"ms_per_step": 1e3 * dt / args.steps, "value": p.dof * args.steps / dt / 1e6,
                 "kernels": kern, "status": mm.STATUS.get(status, status)}
        if prec == "fp64":
            ref = out
        else:
            entry["err_vs_fp64"] = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
        entry["roofline"], _ = roofline(kern, prec, p)
        if not args.no_at_T:
            # the whole interval to T, untimed: error against the FP64 path (whole grid)
            # and against the oracle (its stored samples), and the stated target
            uT, stT = run_to_T(mm, op, p)
            if prec == "fp64":
                ref_T = uT
            else:
                entry["err_at_T_vs_fp64"] = float(np.max(np.abs(uT - ref_T)) / np.max(np.abs(ref_T)))
            if samples is not None:
                mx, idx, val = samples
                entry["err_at_T_vs_oracle_samples"] = float(np.max(np.abs(uT.reshape(-1)[idx] - val)) / mx)
            entry["status_at_T"] = mm.STATUS.get(stT, stT)
            tgt = target(prec)
            if tgt is not None:
                err = entry.get("err_at_T_vs_oracle_samples", entry["err_at_T_vs_fp64"])
                entry["err_at_T"] = max(err, entry["err_at_T_vs_fp64"])
                entry["target"] = tgt
                entry["meets_target"] = bool(entry["err_at_T"] <= tgt and stT == mm.MM_OK)
        if prec == args.headline and args.latency_reps > 0:
            entry["latency"] = latency(mm, ctx, op, p, args.latency_reps)
        op.close()
        res[prec] = entry
        print(f"[bench] {prec}: {entry['ms_per_step']:.3f} ms/step"
              + (f", err at T {entry['err_at_T']:.2e} (target {entry['target']:.0e})" if "err_at_T" in entry else ""),
              file=sys.stderr, flush=True)

    if args.fold != 0:
        # the plain FP64 products on the same workload (timed steps only): the form the
        # mixed precisions are compared with besides the folded default
        print(f"[bench] fp64 plain products: {args.steps} timed steps", file=sys.stderr, flush=True)
        ctx.set_fold(0)
        op, _, dt, kern, status = time_mode(mm, ctx, p, "fp64", args.steps, args.warmup, args.graph_steps)
        op.close()
        ctx.set_fold(args.fold)
        res["fp64_plain"] = {"ms_per_step": 1e3 * dt / args.steps, "value": p.dof * args.steps / dt / 1e6,
                             "kernels": kern, "status": mm.STATUS.get(status, status),
                             "roofline": roofline(kern, "fp64", p)[0]}
        print(f"[bench] fp64 plain products: {res['fp64_plain']['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)

    head = res[args.headline]
    roof, kname = roofline(head["kernels"], args.headline, p)
    roof["traffic"] = measured_traffic() if (kname == "gemm_n" and args.headline == "fp64"
                                             and args.workload == WORKLOAD) else None
    accurate = [m for m, e in res.items() if e.get("meets_target")]
    fastest_accurate = min(accurate, key=lambda m: res[m]["ms_per_step"]) if accurate else None

    line = {
        "metric": "Mdof*steps/s at 256^3 (255^3 interior), FP64 vs MFMA mixed at stated error; p50/p99 solve latency",
        "value": head["value"],
        "unit": "Mdof*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name(args.headline),
        "data": "synthetic",
        "config": {"workload": DESCRIPTION.get(args.workload, args.workload),
                   "dof": p.dof, "scheme": p.scheme, "headline_mode": args.headline,
                   "graph_steps": args.graph_steps, "tile": args.tile or "auto",
                   "sliced_chain": args.sliced_chain, "fold": args.fold,
                   "warmup_min_seconds": WARMUP_MIN_S},
        "latency": head.get("latency"),
        "modes": {m: {kk: vv for kk, vv in e.items() if kk != "kernels"} for m, e in res.items()},
        "fastest_mode_meeting_target": fastest_accurate,
        "speedup_of_that_mode_over_fp64": (res["fp64"]["ms_per_step"] / res[fastest_accurate]["ms_per_step"]
                                           if fastest_accurate else None),
        "speedup_of_that_mode_over_plain_fp64": (res["fp64_plain"]["ms_per_step"] / res[fastest_accurate]["ms_per_step"]
                                                 if fastest_accurate and "fp64_plain" in res else None),
        "kernels": {m: e["kernels"] for m, e in res.items()},
        "roofline": roof,
    }
    serving = {}
    for prec in [m for m in args.serve.split(",") if m]:
        print(f"[bench] served stream: {args.serve_count} requests, {prec}", file=sys.stderr, flush=True)
        serving[prec] = serve_stream(mm, prec, args.serve_count, args.serve_active)
        print(f"[bench] served stream {prec}: p50 {serving[prec]['p50_ms']:.1f} ms "
              f"p99 {serving[prec]['p99_ms']:.1f} ms makespan {serving[prec]['makespan_s']:.2f} s",
              file=sys.stderr, flush=True)
    if serving and not args.no_serial and "fp64" in serving:
        print(f"[bench] served stream: {args.serve_count} requests, fp64, one at a time", file=sys.stderr,
              flush=True)
        serving["fp64_one_at_a_time"] = serve_stream(mm, "fp64", args.serve_count, 1)
        s1, sN = serving["fp64_one_at_a_time"], serving["fp64"]
        serving["batched_over_one_at_a_time"] = {
            "throughput": sN["throughput_mdof_steps_per_s"] / s1["throughput_mdof_steps_per_s"],
            "p50_latency": s1["p50_ms"] / sN["p50_ms"], "p99_latency": s1["p99_ms"] / sN["p99_ms"]}
        print(f"[bench] one at a time: p50 {s1['p50_ms']:.1f} ms p99 {s1['p99_ms']:.1f} ms "
              f"makespan {s1['makespan_s']:.2f} s", file=sys.stderr, flush=True)
    if serving:
        line["serving"] = serving
    if not args.no_configs:
        line["configs"] = config_lines(mm, ctx, args.warmup)
    if not args.no_cpu:
        print(f"[bench] cpu baseline: {args.cpu_steps} oracle steps", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
        if not args.no_configs:
            print("[bench] cpu baselines of the other workloads", file=sys.stderr, flush=True)
            line["cpu_baselines"] = cpu_baselines()
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
