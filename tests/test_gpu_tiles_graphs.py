"""Launch variants that must not change results: the 64- and 128-wide workgroup tiles
of the mode-product kernels, and step loops replayed from recorded HIP graphs.

Both tile sizes sum over k in the same chunk order with the same lane permutation, so
their outputs are bit-for-bit equal in every precision; each is also checked against
the FP64 oracle on ragged shapes that span several tiles of either size. A graph
replays exactly the kernels a direct call launches, so replayed steps are bitwise equal
to directly launched ones; every replay is compared, with unrelated eager work and
synchronisation between replays.
"""
import numpy as np
import pytest

import synth
from oracle import adr, expo

pytestmark = pytest.mark.gpu

U24 = 2.0 ** -24
# per-action bars of the mixed modes (see the mixed-precision tests for the derivation)
ACTION_TOL = {"fp64": 1e-12, "fp32": 3 * (2 * U24 + 16 * U24), "bf16x6": 3 * (2 * U24 + 16 * U24),
              "bf16x3": 3 * (2 * 2.0 ** -16 + 16 * U24)}


@pytest.fixture(scope="module")
def mm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_15861_amd as m
    return m


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


SHAPES = [(9, 13), (200, 130), (5, 6, 7), (70, 65, 66), (130, 129, 127)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("n", SHAPES)
def test_tiles_agree_and_match_oracle(mm, n, prec):
    p = synth.smooth_problem(n, 5, tau=1e-3)
    V = np.random.default_rng(9).standard_normal(p.shape)
    ref = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau).expv(1.0, V)
    got = {}
    for tile in (32, 64, 128):   # 32 applies to FP64; the other precisions take 64 then
        ctx = mm.Context(0)
        ctx.set_gemm_tile(tile)
        op = mm.setup_problem(ctx, p, prec=prec)
        out = dev(np.zeros(p.shape))
        mm.mumode_expv(op, dev(V), out)
        got[tile] = host(out)
        op.close()
        ctx.close()
    assert np.array_equal(got[64], got[128])
    assert np.array_equal(got[32], got[64])
    assert relerr(got[64], ref) <= ACTION_TOL[prec]


def test_bad_tile_rejected(mm):
    ctx = mm.Context(0)
    with pytest.raises(mm.MumodeError):
        ctx.set_gemm_tile(96)
    with pytest.raises(mm.MumodeError):
        ctx.set_graph_steps(-1)
    ctx.close()


GRAPH_CASES = [("le", (63, 63), "fp64"), ("l2b", (20, 17, 15), "fp64"), ("l2b", (24, 20, 18), "bf16x3"),
               ("etd2rk", (19, 16, 14), "fp64"), ("erk2p1f", (33, 31), "fp32")]


@pytest.mark.parametrize("scheme,n,prec", GRAPH_CASES)
def test_graph_replay_equals_direct(mm, scheme, n, prec):
    import torch
    p = synth.smooth_problem(n, 6, tau=1e-3, scheme=scheme, beta=(2.0, -1.0, 0.5)[: len(n)])
    nsteps = 7            # two replays of three steps and one direct step per call
    results = {}
    for gs in (0, 3):
        ctx = mm.Context(0)
        ctx.set_graph_steps(gs)
        op = mm.setup_problem(ctx, p, prec=prec)
        u = dev(p.u0)
        outs = []
        for call in range(3):
            mm.step(op, u, nsteps)
            outs.append(host(u).copy())
            # unrelated eager work and a synchronisation between replays
            w = torch.arange(4096, device="cuda", dtype=torch.float64)
            assert float((w * 2).sum()) == 4096 * 4095
            torch.cuda.synchronize()
        # a second state buffer records the graph again
        u2 = dev(p.u0)
        mm.step(op, u2, nsteps)
        outs.append(host(u2).copy())
        assert mm.mm_check(op) == mm.MM_OK
        op.close()
        ctx.close()
        results[gs] = outs
    for a, b in zip(results[0], results[3]):
        assert np.array_equal(a, b)
    assert np.array_equal(results[3][0], results[3][3])
