"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

- 255^3 Lawson2b, all 100 steps to T = 0.1: FP64 within 1e-12 of the oracle at T, and
  the exact-slice mode with six digits within its stated 1e-9, on the oracle's stored
  samples of u(T) (tests/golden/oracle_3d_n255_l2b_T.txt, written by
  tests/golden/make_oracle_samples.py from oracle/ alone);
- 127^3 Lawson2b, all 200 steps: FP64 within 1e-12 on the stored samples;
- 383^3 ETD2RK with 6-node phi1 and the anisotropic coefficient: one step in FP64
  (1e-12) and with six digits (1e-9), element by element against the oracle's step.
"""
import os

import numpy as np
import pytest

import synth
from oracle import schemes as S

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_15861_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mm):
    c = mm.Context(0)
    yield c
    c.close()


def samples(workload):
    idx, val, mx = [], [], None
    for line in open(os.path.join(GOLDEN, f"oracle_{workload}_T.txt")):
        if line.startswith("#"):
            continue
        a, b = line.split()
        if a == "max_abs":
            mx = float.fromhex(b)
        else:
            idx.append(int(a))
            val.append(float.fromhex(b))
    return mx, np.array(idx), np.array(val)


def solve_on_gpu(mm, ctx, p, prec, steps=None):
    import torch
    print(f"[full size] {p.name} {prec} {steps or p.steps} steps", flush=True)
    op = mm.setup_problem(ctx, p, prec=prec)
    u = torch.from_numpy(p.u0).to("cuda")
    mm.step(op, u, steps or p.steps)
    assert mm.mm_check(op) == mm.MM_OK
    out = u.cpu().numpy()
    op.close()
    return out


@pytest.mark.parametrize("workload,prec,bar", [("3d_n255_l2b", "fp64", 1e-12), ("3d_n255_l2b", "sliced6", 1e-9),
                                               ("3d_n127_l2b", "fp64", 1e-12)])
def test_whole_solve_at_T_on_oracle_samples(mm, ctx, workload, prec, bar):
    p = synth.workload(workload)
    mx, idx, val = samples(workload)
    got = solve_on_gpu(mm, ctx, p, prec)
    assert float(np.max(np.abs(got))) == pytest.approx(mx, rel=bar)
    err = float(np.max(np.abs(got.reshape(-1)[idx] - val)) / mx)
    print(f"{workload} {prec} at T: {err:.2e} on {idx.size} samples (bar {bar:.0e})")
    assert err <= bar


@pytest.fixture(scope="module")
def c5_oracle_step():
    p = synth.workload("3d_n383_etd2rk")
    return p, S.solve(p, steps=1)


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("sliced6", 1e-9)])
def test_383_etd2rk_step(mm, ctx, c5_oracle_step, prec, bar):
    p, ref = c5_oracle_step
    got = solve_on_gpu(mm, ctx, p, prec, steps=1)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"383^3 ETD2RK q = 6, one step, {prec}: {err:.2e} (bar {bar:.0e})")
    assert err <= bar
