"""The 2D experiment of Sec. 4.2 at the 512 x 512 configuration (16 separable
sine modes plus white noise of standard deviation 0.1, x0 = 0, 32 x 32 tiles
without overlap, to relative residual 1e-6): on every seed and s the GPU
solve stops at the oracle's cycle (classical Jacobi: sweep), with the
oracle's residual, and its iterate equals the oracle's bit for bit at 64
fixed points.  The oracle's results are stored in
tests/golden/c2_poisson2d_512.json by tests/golden/make_c2_golden.py (which
calls only the oracle): the full oracle solves take minutes of CPU time."""
import json
import os

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_poisson2d_512.json")


def _cases():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    return g, [(c["seed"], c["method"]) for c in g["cases"]]


_G, _IDS = _cases()


@pytest.mark.parametrize("seed,method", _IDS)
def test_c2_solve_to_tolerance_matches_oracle(seed, method):
    case = next(c for c in _G["cases"] if c["seed"] == seed and c["method"] == method)
    f, h = W.make("poisson2d_512", seed)
    F = torch.from_numpy(f).cuda()
    X = torch.zeros_like(F)
    if method == "classical":
        info = hj.solve_2d(F, X, h, method="global", rel_tol=_G["tol"], max_cycles=10_000_000)
    else:
        info = hj.solve_2d(F, X, h, tile=tuple(_G["tile"]), s=case["s"], overlap=tuple(_G["overlap"]),
                           rel_tol=_G["tol"], max_cycles=10_000_000)
    print(f"c2 seed {seed} {method}: gpu {info.cycles} cycles, oracle {case['cycles']}", flush=True)
    assert info.cycles == case["cycles"]
    assert abs(info.rel_residual - case["rel_residual"]) <= 1e-9 * case["rel_residual"]
    x = X.cpu().numpy()
    got = np.array([x[r, c] for r, c in _G["points"]])
    want = np.array([float.fromhex(v) for v in case["values_hex"]])
    assert np.array_equal(got, want)
