"""The allocation-free exponential action (mumode_expv_noalloc) against mumode_expv: two
calls in a row on one device, the second on a smaller grid, each bit-identical to the
operator-based action with the same factors (and within 1e-12 of the oracle); a grid
beyond the scratch limit is refused before any launch."""
import numpy as np
import pytest

import synth
from oracle import adr, expo

pytestmark = pytest.mark.gpu


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


def test_noalloc_matches_expv_twice(mm):
    import torch
    ctx = mm.Context(0)
    try:
        for n, seed in (((61, 70, 45), 3), ((33, 20), 4)):
            print(f"[noalloc] grid {n}", flush=True)
            p = synth.smooth_problem(n, seed, tau=1e-3, beta=(4.0,) * len(n))
            op = mm.setup_problem(ctx, p)
            x = dev(p.u0)
            ref = torch.empty_like(x)
            mm.mumode_expv(op, x, ref)
            factors = [dev(op.factor(mu, 0)) for mu in range(p.d)]
            out = torch.full_like(x, np.nan)
            mm.mumode_expv_noalloc(ctx, factors, x, out)
            got, want = host(out), host(ref)
            assert np.array_equal(got, want)
            orc = expo.KronOperator(p.n, adr.extracted_amax(p.a), p.lam, p.beta_bar, p.tau).expv(1.0, p.u0)
            assert float(np.max(np.abs(got - orc)) / np.max(np.abs(orc))) <= 1e-12
            # in place (in and out alias)
            mm.mumode_expv_noalloc(ctx, factors, x, x)
            assert np.array_equal(host(x), want)
            op.close()
    finally:
        ctx.close()


def test_noalloc_refuses_grids_beyond_the_scratch(mm):
    import torch
    ctx = mm.Context(0)
    try:
        n = 129                      # 129^3 > 2^21
        f = torch.eye(n, dtype=torch.float64, device="cuda")
        x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        with pytest.raises(mm.MumodeError, match="scratch limit"):
            mm.mumode_expv_noalloc(ctx, [f, f, f], x, x)
    finally:
        ctx.close()
