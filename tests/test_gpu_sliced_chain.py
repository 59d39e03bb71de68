"""Chained exact-slice actions of Lawson steps against the unchained sliced path.

In the chained form every mode product but the last writes the next product's digit
planes and fiber exponents from its own epilogue (a workgroup covers whole fibers of the
next product), instead of writing FP64 values that a separate split pass reads back. The
fiber exponents are the maxima of the same FP64 values and the digits the same bytes, and
the integer level sums do not depend on the order of k, so both forms give the same bits.
The unchained path is checked against the sliced and exact oracles elsewhere; here every
case must agree with it exactly, over several steps (so that the second step starts from
a state the first chained action produced), and the default mode uses the chain at the
255^3 size (the full-size accuracy tests at T then run through it).
"""
import numpy as np
import pytest

import synth

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
    c.set_sliced_chain(1)
    c.close()


def run(mm, ctx, p, prec, mode, steps):
    import torch
    ctx.set_sliced_chain(mode)
    op = mm.setup_problem(ctx, p, prec=prec)
    u = torch.from_numpy(p.u0.copy()).to("cuda")
    mm.lawson_step(op, u, steps)
    torch.cuda.synchronize()
    assert mm.mm_check(op) == mm.MM_OK
    got = u.cpu().numpy()
    op.close()
    return got


# (grid n1, n2[, n3], digits S, scheme, chain mode, steps): 3D and 2D, axes shorter and
# longer than 128 (mode 2 forces the chain on short axes), both workgroup shapes
CASES = [((200, 150, 130), 5, "l2b", 2, 3), ((130, 255, 140), 6, "le", 2, 3), ((64, 40, 33), 4, "l2b", 2, 2),
         ((64, 40, 33), 7, "le", 3, 2), ((150, 131, 256), 3, "l2b", 3, 2), ((255, 200), 6, "l2b", 2, 3),
         ((33, 250), 7, "le", 3, 3), ((256, 1), 5, "l2b", 2, 2), ((1, 1, 1), 6, "l2b", 2, 2)]


@pytest.mark.parametrize("n,S,scheme,mode,steps", CASES)
def test_chain_equals_unchained(mm, ctx, n, S, scheme, mode, steps):
    p = synth.smooth_problem(n, 21, tau=1e-3, scheme=scheme)
    ref = run(mm, ctx, p, f"sliced{S}", 0, steps)
    got = run(mm, ctx, p, f"sliced{S}", mode, steps)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))


def test_chain_full_size_default_mode(mm, ctx):
    """255^3 Lawson2b, sliced6, two steps: the default mode (which takes the chain at this
    size) agrees bit for bit with the unchained path, and so do the four-wave workgroups."""
    p = synth.workload("3d_n255_l2b")
    ref = run(mm, ctx, p, "sliced6", 0, 2)
    got = run(mm, ctx, p, "sliced6", 1, 2)
    assert np.array_equal(got, ref)
    wide = run(mm, ctx, p, "sliced6", 3, 2)
    assert np.array_equal(wide, ref)


def test_chain_mode_validation(mm, ctx):
    with pytest.raises(mm.MumodeError):
        ctx.set_sliced_chain(4)
    with pytest.raises(mm.MumodeError):
        ctx.set_sliced_chain(-1)
    ctx.set_sliced_chain(1)
