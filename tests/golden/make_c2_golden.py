"""Write tests/golden/c2_poisson2d_512.json: the oracle's cycles to a relative
residual of 1e-6 on the 512 x 512 workload (16 separable sine modes plus white
noise of standard deviation 0.1, x0 = 0), 32 x 32 tiles without overlap (the
2D experiment of Sec. 4.2) for s in {1, 4, 8, 16, 32} and for classical
Jacobi, seeds 0-2, with the final relative residual and the exact values of
the returned iterate at 64 fixed points.  Calls only oracle/ (and the seeded
input generator).

    PYTHONPATH=. python tests/golden/make_c2_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_16465_amd import workloads as W  # noqa: E402

N, TOL, TILE = 512, 1e-6, (32, 32)
S_GRID = (1, 4, 8, 16, 32)
SEEDS = (0, 1, 2)


def sample_points(n, k=64, seed=123):
    rng = np.random.default_rng(seed)
    return [[int(r), int(c)] for r, c in zip(rng.integers(0, n, k), rng.integers(0, n, k))]


def main():
    pts = sample_points(N)
    out = {"description": __doc__.split("\n\n")[0].replace("\n", " "),
           "n": N, "tol": TOL, "tile": list(TILE), "overlap": [0, 0], "points": pts, "cases": []}
    for seed in SEEDS:
        f, h = W.make("poisson2d_512", seed)
        x0 = np.zeros_like(f)
        runs = [("classical", oracle.CLASSICAL, 1)] + [(f"s{s}", oracle.HIERARCHICAL, s) for s in S_GRID]
        for name, method, s in runs:
            t = time.time()
            x, cycles, rel, r0 = oracle.solve_2d(f, x0, h, h, method=method, tile=TILE, s=s, tol=TOL,
                                                 max_cycles=10**7)
            vals = [float(x[r, c]).hex() for r, c in pts]
            out["cases"].append({"seed": seed, "method": name, "s": s, "cycles": cycles,
                                 "rel_residual": rel, "r0_norm": r0, "values_hex": vals})
            print(f"seed {seed} {name}: {cycles} cycles, rel {rel:.6e} ({time.time() - t:.1f} s)", flush=True)
    with open(os.path.join(HERE, "c2_poisson2d_512.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
