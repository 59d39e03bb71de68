"""Benchmark: Mdof*steps/s of the mu-mode Lawson2b path on the 255^3 workload.

One step = one Lawson2b step over the whole grid: two fused remainder/stage passes and
one stacked exp action (three mode products on two grid functions). The workload is the
3D Dirichlet ADR problem with 255^3 interior points (h = 1/256), a = 1 + 0.9 tanh(s),
beta = (10, 10, 10), r = u^2(1 - u), tau = 1e-3, 100 steps to T = 0.1 (synthetic seeded
inputs). Every contraction precision is timed; the headline value is the FP64 path
unless --headline names another mode. Each mixed mode's error is reported against the
FP64 path after the same steps (the FP64 path matches the CPU oracle to 1e-12 in the
parity tests).

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
HBM_PEAK = 8.0e12
WORKLOAD = "3d_n255_l2b"


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
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--serve", default="fp64,bf16x3",
                    help="precisions for the served-stream run ('' to skip)")
    ap.add_argument("--serve-count", type=int, default=512)
    ap.add_argument("--serve-active", type=int, default=16)
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


def dtype_name(prec):
    """Arithmetic type of a mode's contractions."""
    if prec.startswith("sliced"):
        return f"i8x{prec[6:]}"          # S int8 digit planes, int32 accumulation, f64 combination
    return {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3", "bf16x6": "bf16x6"}[prec]


def slice_products(prec):
    S = int(prec[6:])
    return S * (S + 1) // 2


def time_mode(mm, ctx, p, prec, steps, warmup, graph_steps=0):
    """Timed region: `steps` steps on a resident state, no per-kernel events. A second,
    untimed pass of the same steps brackets every kernel with HIP events on its stream
    for the per-kernel table and the roofline. With graph replay the warmup runs at
    least one graph's worth of steps, so that the graph is recorded before timing."""
    import torch
    op = mm.setup_problem(ctx, p, prec=prec)
    u0 = torch.from_numpy(p.u0).to("cuda")
    u = u0.clone()
    stream = torch.cuda.current_stream()
    warmup = max(warmup, graph_steps)
    if warmup:
        mm.step(op, u, warmup, stream)
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
            st, u, info = mm.solve_poll(srv, rid, p.shape)
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
    srv.close()
    lat = np.array(lat) * 1e3
    span = max(done) - t_first
    return {"requests": count, "max_active": max_active, "status": statuses,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": span,
            "throughput_mdof_steps_per_s": work / span / 1e6}


def cpu_baseline(p, steps):
    """The oracle, untuned, on the host cores: `steps` steps of the workload's scheme."""
    import synth
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_limits
        ctxm = threadpool_limits(limits=cores)
    except Exception:  # pragma: no cover
        ctxm = None
    if any(b == synth.PERIODIC for b in getattr(p, "bc", ())):
        from oracle import spectral as S       # periodic pseudo-spectral problems
    elif any(getattr(p, "bc", ())) or getattr(p, "form", "flux") != "flux":
        from oracle import adr3d as S          # Neumann axes or the non-divergence form
    else:
        from oracle import schemes as S
    t0 = time.perf_counter()
    S.solve(p, steps=steps)
    dt = time.perf_counter() - t0
    if ctxm is not None:
        ctxm.unregister() if hasattr(ctxm, "unregister") else None
    return {"value": p.dof * steps / dt / 1e6, "unit": "Mdof*steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} {p.scheme} steps of the {p.name} workload (numpy FP64, OpenBLAS threads = cores)",
            "seconds": dt}


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
    modes = [m for m in args.modes.split(",") if m]
    if "fp64" not in modes:
        modes = ["fp64"] + modes
    res = {}
    ref = None
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
        if prec == args.headline and args.latency_reps > 0:
            entry["latency"] = latency(mm, ctx, op, p, args.latency_reps)
        op.close()
        res[prec] = entry
        print(f"[bench] {prec}: {entry['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)

    head = res[args.headline]
    # roofline of the dominant kernel of the headline mode
    kname = max(("gemm_k", "gemm_n", "stencil", "fused"), key=lambda k: head["kernels"][k]["total_ms"])
    k = head["kernels"][kname]
    if kname == "fused":
        # one workgroup on one compute unit: its share of the FP64 matrix peak
        achieved = k["work"] / (k["total_ms"] * 1e-3)
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["fp64"] / 256 / 1e12,
                "unit": "TFLOP/s", "scope": "one compute unit"}
    elif kname == "stencil":
        # algorithmic bytes per grid point of the fused remainder passes: read u and a,
        # write two outputs (first pass) or read u, a, W and write u (second pass): 32 B
        achieved = 32.0 * k["work"] / (k["total_ms"] * 1e-3)
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    else:
        dtype_peak = {"fp64": "fp64", "fp32": "fp32"}.get(args.headline, "bf16")
        if args.headline.startswith("sliced"):
            # int8 digit products actually executed: S(S+1)/2 per algorithmic multiply-add
            achieved = k["work"] * slice_products(args.headline) / (k["total_ms"] * 1e-3)
            roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK["int8"] / 1e12,
                    "unit": "TOP/s"}
        elif dtype_peak == "bf16":
            # split-BF16 contractions are bound by HBM: 16 B per grid point per pass
            flops_per_point = 2.0 * p.n[0]
            bytes_ = 16.0 * k["work"] / flops_per_point
            achieved = bytes_ / (k["total_ms"] * 1e-3)
            roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
        else:
            achieved = k["work"] / (k["total_ms"] * 1e-3)
            roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[dtype_peak] / 1e12,
                    "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = {"gemm_k": "gemm (mode 1)", "gemm_n": "gemm (modes 2, 3)", "stencil": "stencil",
                      "fused": "whole small-2D solve in one workgroup (one compute unit)"}[kname]
    roof["avg_launch_us"] = k["avg_us"]
    roof["traffic"] = measured_traffic() if (kname == "gemm_n" and args.headline == "fp64"
                                             and args.workload == WORKLOAD) else None

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
                   "graph_steps": args.graph_steps, "tile": args.tile or "auto"},
        "latency": head.get("latency"),
        "modes": {m: {kk: vv for kk, vv in e.items() if kk != "kernels"} for m, e in res.items()},
        "kernels": {m: e["kernels"] for m, e in res.items()},
        "roofline": roof,
    }
    serving = {}
    for prec in [m for m in args.serve.split(",") if m]:
        print(f"[bench] served stream: {args.serve_count} requests, {prec}", file=sys.stderr, flush=True)
        serving[prec] = serve_stream(mm, prec, args.serve_count, args.serve_active)
        print(f"[bench] served stream {prec}: p50 {serving[prec]['p50_ms']:.1f} ms "
              f"p99 {serving[prec]['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    if serving:
        line["serving"] = serving
    if not args.no_cpu:
        print(f"[bench] cpu baseline: {args.cpu_steps} oracle steps", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_steps)
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
