"""Grouped Lawson steps (lawson_step_batch): up to eight problems of one class -- equal
grid, precision, digit count and scheme, each with its own coefficient, velocity,
reaction, tau and state -- advance together, one stencil launch per pass and one grouped
mode product per axis. Every problem's result must equal lawson_step on that problem
alone bit for bit, and the FP64 oracle within 1e-12 (the sliced mode: within its stated
1e-9)."""
import numpy as np
import pytest

import synth
from oracle import adr3d
from oracle import schemes as S

pytestmark = pytest.mark.gpu


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


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def family(n, count, scheme="l2b", steps=6):
    """count problems of one grid with different fields, velocities, reactions and tau."""
    out = []
    for i in range(count):
        d = len(n)
        beta = tuple(float(x) for x in np.random.default_rng(500 + i).uniform(-15, 15, size=d))
        r = synth.R_CUBIC if i % 2 else synth.R_LOGISTIC
        out.append(synth.smooth_problem(n, 100 + i, tau=(1.0 + 0.25 * i) * 1e-3, steps=steps, scheme=scheme,
                                        beta=beta, r=r))
    return out


def run_group(mm, ctx, probs, prec="fp64", steps=None):
    """Grouped solve and each problem alone; returns (grouped, alone) host arrays."""
    ops = [mm.setup_problem(ctx, p, prec=prec) for p in probs]
    us = [dev(p.u0) for p in probs]
    nsteps = steps if steps is not None else probs[0].steps
    print(f"[group] {len(probs)} x {probs[0].n} {prec} {probs[0].scheme} {nsteps} steps", flush=True)
    mm.lawson_step_batch(ops, us, nsteps)
    grouped = [host(u) for u in us]
    alone = []
    for op, p in zip(ops, probs):
        u = dev(p.u0)
        mm.lawson_step(op, u, nsteps)
        assert mm.mm_check(op) == mm.MM_OK
        alone.append(host(u))
    for op in ops:
        op.close()
    return grouped, alone


@pytest.mark.parametrize("n,count", [((40, 33, 28), 5), ((127, 90), 3), ((17, 70, 9), 8), ((63, 63), 4)])
def test_group_equals_alone_and_oracle(mm, ctx, n, count):
    probs = family(n, count)
    grouped, alone = run_group(mm, ctx, probs)
    for g, a, p in zip(grouped, alone, probs):
        assert np.array_equal(g, a)
        assert relerr(g, S.solve(p)) <= 1e-12


def test_lawson_euler_group(mm, ctx):
    probs = family((30, 31, 32), 3, scheme="le")
    grouped, alone = run_group(mm, ctx, probs)
    for g, a, p in zip(grouped, alone, probs):
        assert np.array_equal(g, a)
        assert relerr(g, S.solve(p)) <= 1e-12


def test_small_2d_group_runs_one_workgroup_each(mm, ctx):
    """63 x 63 FP64 problems take the one-workgroup solver, one workgroup per problem."""
    probs = family((63, 63), 7, steps=30)
    ctx.timing(True)
    grouped, alone = run_group(mm, ctx, probs)
    launches, _, _ = ctx.timing_read(mm.MM_KIND_FUSED)
    ctx.timing(False)
    assert launches == 1 + len(probs)   # the grouped launch, then one per problem alone
    for g, a, p in zip(grouped, alone, probs):
        assert np.array_equal(g, a)
        assert relerr(g, S.solve(p)) <= 1e-12


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "sliced6"])
def test_group_other_precisions(mm, ctx, prec):
    probs = family((36, 30, 33), 4)
    grouped, alone = run_group(mm, ctx, probs, prec=prec)
    for g, a, p in zip(grouped, alone, probs):
        assert np.array_equal(g, a)
        if prec == "sliced6":
            assert relerr(g, S.solve(p)) <= 1e-9


def test_neumann_nondivergence_group(mm, ctx):
    """The problem of Sec. 5.2 (Neumann faces at x = 1, a Lap u, advection in A) at two
    velocities: one class, two operators."""
    probs = [synth.paper3d_problem(16, b, 1.0, scheme="l2b", steps=32) for b in (-0.01, -1.0)]
    grouped, alone = run_group(mm, ctx, probs)
    for g, a, p in zip(grouped, alone, probs):
        assert np.array_equal(g, a)
        assert relerr(g, adr3d.solve(p)) <= 1e-12


def test_group_refuses_mixed_classes(mm, ctx):
    p1 = synth.smooth_problem((20, 18, 16), 1, tau=1e-3, steps=2)
    p2 = synth.smooth_problem((20, 18, 17), 2, tau=1e-3, steps=2)
    o1, o2 = mm.setup_problem(ctx, p1), mm.setup_problem(ctx, p2)
    o3 = mm.setup_problem(ctx, p1, prec="fp32")
    u1, u2 = dev(p1.u0), dev(p2.u0)
    with pytest.raises(mm.MumodeError, match="EINVAL"):
        mm.lawson_step_batch([o1, o2], [u1, u2], 1)          # different grids (checked in C)
    with pytest.raises(mm.MumodeError, match="EINVAL"):
        mm.lawson_step_batch([o1, o3], [u1, dev(p1.u0)], 1)  # different precisions
    with pytest.raises(mm.MumodeError, match="EINVAL"):
        mm.lawson_step_batch([o1, o1], [u1, dev(p1.u0)], 1)  # one operator twice
    for o in (o1, o2, o3):
        o.close()
