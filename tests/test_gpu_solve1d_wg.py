"""GPU parity of the one-workgroup 1D solve (small hierarchical 1D problems
run all their cycles inside one workgroup).  It must give the same iterates,
bit for bit, as one launch per cycle and as the CPU FP64 oracle, stop at the
same cycle, and report the same status; residual norms agree to rounding
(the reductions sum in a different order)."""
import sys

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (n, tile, s, overlap): 5 tiles (the paper's 1D size with exact-regime
# overlap), 16 tiles (the most one workgroup holds, ragged last tile), a grid
# shorter than the tile, 2, 6 and 11 tiles; f and both iterates take 60 KiB
# of LDS at n = 2560 and 117 KiB at n = 5000 (above the 64 KiB a workgroup
# gets without opting in).
SHAPES = [(256, 64, 8, 14), (1000, 64, 8, 0), (37, 64, 5, 0), (700, 128, 6, 10), (300, 256, 3, 0),
          (2560, 512, 24, 46), (5000, 512, 24, 46)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    hj.load()
    yield


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def both(f, x0, h, dtype=torch.float64, **kw):
    """(x, info) from the one-workgroup solve and from one launch per cycle."""
    out = []
    for per_cycle in (False, True):
        X = dev(x0, dtype)
        info = hj.solve_1d(dev(f, dtype), X, h, allow_not_converged=True, launch_per_cycle=per_cycle, **kw)
        out.append((host(X), info))
    return out


@pytest.mark.parametrize("n,tile,s,ov", SHAPES)
def test_wg_fixed_cycles_match_oracle_and_per_cycle_launches(orc, n, tile, s, ov):
    f = W.rhs_1d_modes(n, 8, 5)
    h = 1.0 / (n + 1)
    x0 = W.rhs_1d_modes(n, 3, 6)  # a non-zero start exercises the halo reads of cycle 0
    for nc in (1, 2, 7, 33):
        say(f"wg fixed n={n} tile={tile} s={s} ov={ov} cycles={nc}")
        (xw, iw), (xp, ip) = both(f, x0, h, tile=tile, s=s, overlap=ov, rel_tol=0.0, max_cycles=nc)
        assert iw.cycles == ip.cycles == nc and iw.sweeps == nc * s
        assert np.array_equal(xw, xp)
        assert np.array_equal(xw, orc.hier_1d(f, x0, h, tile, s, nc, ov))
        assert abs(iw.rel_residual - ip.rel_residual) <= 1e-13 * ip.rel_residual
        assert abs(iw.r0_norm - ip.r0_norm) <= 1e-13 * ip.r0_norm


@pytest.mark.parametrize("n,tile,s,ov", SHAPES)
def test_wg_to_tolerance_matches_oracle(orc, n, tile, s, ov):
    f = W.rhs_1d_modes(n, 8, 9)
    h = 1.0 / (n + 1)
    x0 = np.zeros(n)
    say(f"wg to tol n={n} tile={tile} s={s} ov={ov}")
    (xw, iw), (xp, ip) = both(f, x0, h, tile=tile, s=s, overlap=ov, rel_tol=1e-6)
    xo, co, relo, r0o = orc.solve_1d(f, x0, h, tile=tile, s=s, tol=1e-6, overlap=ov)
    assert iw.status == ip.status == hj.HJ_OK
    assert iw.cycles == ip.cycles == co > 0
    assert np.array_equal(xw, xp) and np.array_equal(xw, xo)
    assert abs(iw.rel_residual - relo) <= 1e-12 * relo
    assert abs(iw.r0_norm - r0o) <= 1e-12 * r0o


def test_wg_fp32_matches_per_cycle_launches():
    """FP32 near the largest grid one workgroup holds (15 tiles of 512)."""
    n, tile, s, ov = 7000, 512, 8, 14
    f = W.rhs_1d_modes(n, 8, 2)
    h = 1.0 / (n + 1)
    say(f"wg fp32 n={n}")
    for kw in (dict(rel_tol=0.0, max_cycles=40), dict(rel_tol=1e-4)):
        (xw, iw), (xp, ip) = both(f, np.zeros(n), h, torch.float32, tile=tile, s=s, overlap=ov, **kw)
        assert iw.cycles == ip.cycles > 0
        assert np.array_equal(xw, xp)


def test_wg_chunks_and_cycle_cap_match_per_cycle_launches():
    """More cycles than one launch runs (4096): fixed count across chunk
    boundaries, and a tolerance the cap stops short of (not converged)."""
    n, tile, s = 256, 64, 1
    f = W.rhs_1d_modes(n, 8, 1)
    h = 1.0 / (n + 1)
    for kw, status in ((dict(rel_tol=0.0, max_cycles=9000), hj.HJ_OK),
                       (dict(rel_tol=1e-14, max_cycles=8193), hj.HJ_ERR_NOT_CONVERGED)):
        say(f"wg chunks {kw}")
        (xw, iw), (xp, ip) = both(f, np.zeros(n), h, tile=tile, s=s, **kw)
        assert iw.status == ip.status == status
        assert iw.cycles == ip.cycles == kw["max_cycles"]
        assert np.array_equal(xw, xp)
        assert abs(iw.rel_residual - ip.rel_residual) <= 1e-12 * ip.rel_residual


def test_wg_nonfinite_input_stops_like_per_cycle_launches():
    n = 256
    f = W.rhs_1d_modes(n, 8, 3)
    f[100] = np.nan
    h = 1.0 / (n + 1)
    say("wg nonfinite")
    for per_cycle in (False, True):
        with pytest.raises(hj.HJError) as e:
            hj.solve_1d(dev(f), dev(np.zeros(n)), h, tile=64, s=8, overlap=14, rel_tol=1e-6,
                        launch_per_cycle=per_cycle)
        assert e.value.status == hj.HJ_ERR_NONFINITE


def _batch_specs(count, seed):
    rng = np.random.default_rng(seed)
    return [(int(n), W.rhs_1d_modes(int(n), 8, 100 + i)) for i, n in enumerate(rng.integers(37, 2501, count))]


@pytest.mark.parametrize("mode", ["to_tol", "fixed", "capped"])
def test_wg_batch_matches_single_solves_and_oracle(orc, mode):
    """HJ_BATCH_WG1D: ragged 1D sizes (37..2500 points, 1 to 11 tiles of 256,
    s = 16, overlap 30), one workgroup per problem; every problem's iterate
    and info equal its own hj_solve_1d call, and the oracle's."""
    specs = _batch_specs(24, 4)
    kw = {"to_tol": dict(rel_tol=1e-6, max_cycles=100_000),
          "fixed": dict(rel_tol=0.0, max_cycles=7),
          "capped": dict(rel_tol=1e-9, max_cycles=5)}[mode]
    shape = dict(tile_1d=256, s_1d=16, overlap_1d=30)
    say(f"wg batch {mode}: {len(specs)} problems")
    Fs = [dev(f) for _, f in specs]
    Xs = [dev(np.zeros(n)) for n, _ in specs]
    infos = hj.solve_batched([(F, X, 1.0 / (n + 1)) for F, X, (n, _) in zip(Fs, Xs, specs)],
                             one_workgroup_1d=True, allow_not_converged=True, **shape, **kw)
    for i, ((n, f), F, X, ib) in enumerate(zip(specs, Fs, Xs, infos)):
        X1 = dev(np.zeros(n))
        i1 = hj.solve_1d(F, X1, 1.0 / (n + 1), tile=256, s=16, overlap=30, allow_not_converged=True, **kw)
        assert ib.cycles == i1.cycles and ib.sweeps == i1.sweeps, i
        assert ib.status == i1.status, i
        assert np.array_equal(host(X), host(X1)), i
        assert abs(ib.rel_residual - i1.rel_residual) <= 1e-13 * i1.rel_residual, i
        if mode == "capped":
            assert ib.cycles == 5 and ib.status == hj.HJ_ERR_NOT_CONVERGED
        if i < 4:
            h = 1.0 / (n + 1)
            if mode == "fixed":
                want = orc.hier_1d(f, np.zeros(n), h, 256, 16, 7, 30)
            else:
                want, co, _, _ = orc.solve_1d(f, np.zeros(n), h, tile=256, s=16, tol=kw["rel_tol"],
                                              overlap=30, max_cycles=kw["max_cycles"])
                assert ib.cycles == (co if co >= 0 else kw["max_cycles"]), i
            assert np.array_equal(host(X), want), i


def test_wg_batch_rejects_what_one_workgroup_cannot_hold():
    n = 256
    f = dev(W.rhs_1d_modes(n, 8, 0))
    prob = [(f, dev(np.zeros(n)), 1.0 / (n + 1))]
    for kw in (dict(tile_1d=32, s_1d=8, overlap_1d=0),         # LDS tile body
               dict(tile_1d=64, s_1d=8, overlap_1d=0, autotune=True)):
        with pytest.raises(hj.HJError) as e:
            hj.solve_batched(prob, one_workgroup_1d=True, **kw)
        assert e.value.status == hj.HJ_ERR_UNSUPPORTED
    big = 7000  # 3 n 8 B > 150 KiB
    fb = dev(W.rhs_1d_modes(big, 8, 0))
    with pytest.raises(hj.HJError) as e:
        hj.solve_batched([(fb, dev(np.zeros(big)), 1.0 / (big + 1))], one_workgroup_1d=True,
                         tile_1d=512, s_1d=8, overlap_1d=14)
    assert e.value.status == hj.HJ_ERR_UNSUPPORTED
    f2 = dev(W.rhs_2d_modes(64, 64, 4, 0.0, 0))
    with pytest.raises(hj.HJError) as e:
        hj.solve_batched([(f2, dev(np.zeros((64, 64))), 1.0 / 65)], one_workgroup_1d=True, tile=(32, 32), s=4,
                         overlap=(0, 0))
    assert e.value.status == hj.HJ_ERR_UNSUPPORTED


def test_wg_batch_fp32_matches_single_solves():
    """FP32 batch (37..2500 points, at most 10 tiles of 256): each problem
    equals its own FP32 hj_solve_1d call bit for bit."""
    specs = _batch_specs(8, 7)
    say(f"wg batch fp32: {len(specs)} problems")
    Fs = [dev(f, torch.float32) for _, f in specs]
    Xs = [dev(np.zeros(n), torch.float32) for n, _ in specs]
    infos = hj.solve_batched([(F, X, 1.0 / (n + 1)) for F, X, (n, _) in zip(Fs, Xs, specs)], rel_tol=1e-4,
                             max_cycles=100_000, tile_1d=256, s_1d=8, overlap_1d=14, one_workgroup_1d=True,
                             allow_not_converged=True)
    for i, ((n, _), F, X, ib) in enumerate(zip(specs, Fs, Xs, infos)):
        assert hj.axis_tiles(n, 256, 14) <= 16
        X1 = dev(np.zeros(n), torch.float32)
        i1 = hj.solve_1d(F, X1, 1.0 / (n + 1), tile=256, s=8, overlap=14, rel_tol=1e-4, max_cycles=100_000,
                         allow_not_converged=True)
        assert ib.cycles == i1.cycles and ib.status == i1.status, i
        assert np.array_equal(host(X), host(X1)), i
