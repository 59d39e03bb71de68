"""Write the oracle's solution at the final time T of a named workload, sampled, to a
text fixture (tests/golden/oracle_<workload>_T.txt). Calls only oracle/ and the seeded
input generators; nothing from the GPU path.

    python tests/golden/make_oracle_samples.py 3d_n255_l2b [--samples 4096]

The fixture holds max |u(T)| over the whole grid (the norm of the relative error) and
u(T) at seeded sample points (flat C-order indices), full precision.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import schemes  # noqa: E402


def sample_indices(dof: int, count: int, seed: int = 20250601) -> np.ndarray:
    """Seeded sample of flat grid indices (sorted, distinct), plus the first and last."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(dof, size=min(count, dof), replace=False)
    return np.unique(np.concatenate([idx, [0, dof - 1]]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--samples", type=int, default=4096)
    args = ap.parse_args()
    p = synth.workload(args.workload)
    t0 = time.perf_counter()
    u = schemes.solve(p)
    dt = time.perf_counter() - t0
    flat = u.reshape(-1)
    idx = sample_indices(flat.size, args.samples)
    path = os.path.join(HERE, f"oracle_{args.workload}_T.txt")
    with open(path, "w") as f:
        f.write(f"# oracle solution at T of workload {args.workload} ({p.scheme}, {p.steps} steps of tau = {p.tau}),\n")
        f.write(f"# written by tests/golden/make_oracle_samples.py (oracle/ only; {dt:.0f} s on the host)\n")
        f.write(f"max_abs {float(np.max(np.abs(flat))).hex()}\n")
        for i in idx:
            f.write(f"{int(i)} {float(flat[i]).hex()}\n")
    print(f"wrote {path}: {idx.size} samples, {dt:.1f} s")


if __name__ == "__main__":
    main()
