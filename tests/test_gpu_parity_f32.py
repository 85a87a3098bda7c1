"""GPU parity of the FP32 instantiation against the oracle's FP32 sweeps and
cycles (orc_*_f32, pinned in tests/test_oracle_f32_pins.py), bit for bit:
2D register-resident and LDS tiles, isotropic and anisotropic spacing,
several sub-iteration counts (both paths of the register tile's
two-sweeps-per-trip loop), classical sweeps, 1D register and LDS tiles
(launched per cycle and inside one workgroup), and batches."""
import sys

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
F32 = torch.float32


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dtype=F32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host32(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("tile", [(32, 32), (64, 32), (64, 64), (32, 64), (64, 128), (128, 64), (16, 16)])
@pytest.mark.parametrize("aniso", [False, True])
def test_fp32_2d_cycles_equal_fp32_oracle(orc, tile, aniso):
    ny, nx = 150, 200
    hx = 1.0 / (nx + 1)
    hy = hx * (1.3 if aniso else 1.0)
    f = W.rhs_random((ny, nx), tile[0] + 3 * tile[1] + aniso)
    x0 = W.rhs_random((ny, nx), tile[0] + 3 * tile[1] + aniso + 1)
    for s, ov, nc in ((1, (0, 0), 3), (2, (2, 2), 2), (5, (8, 8), 3), (8, (14, 6), 2)):
        want = orc.hier_2d_f32(f, x0, hx, hy, tile, s, nc, ov)
        for lds in ((False, True) if max(tile) <= 64 else (False,)):
            say(f"fp32 2d tile={tile} aniso={aniso} s={s} ov={ov} lds={lds}")
            X = dev(x0)
            info = hj.solve_2d(dev(f), X, hx=hx, hy=hy, tile=tile, s=s, overlap=ov, rel_tol=0.0, max_cycles=nc,
                               lds_kernel=lds)
            assert info.cycles == nc
            got = host32(X)
            assert got.dtype == np.float32
            assert np.array_equal(got, want), (tile, aniso, s, ov, lds)


@pytest.mark.parametrize("aniso", [False, True])
def test_fp32_classical_sweeps_equal_fp32_oracle(orc, aniso):
    ny, nx = 97, 130
    hx = 1.0 / (nx + 1)
    hy = hx * (0.8 if aniso else 1.0)
    f, x0 = W.rhs_random((ny, nx), 21), W.rhs_random((ny, nx), 22)
    X = dev(x0)
    hj.solve_2d(dev(f), X, hx=hx, hy=hy, method="global", rel_tol=0.0, max_cycles=9)
    assert np.array_equal(host32(X), orc.jacobi_2d_f32(f, x0, hx, hy, 9))
    f1, x1 = W.rhs_random(1000, 23), W.rhs_random(1000, 24)
    X1 = dev(x1)
    hj.solve_1d(dev(f1), X1, 1.0 / 1001, method="global", rel_tol=0.0, max_cycles=9, launch_per_cycle=True)
    assert np.array_equal(host32(X1), orc.jacobi_1d_f32(f1, x1, 1.0 / 1001, 9))


@pytest.mark.parametrize("n,tile,ov", [(1000, 32, 4), (1000, 64, 10), (3000, 256, 30), (37, 64, 0), (5000, 512, 46)])
@pytest.mark.parametrize("launch_per_cycle", [False, True])
def test_fp32_1d_cycles_equal_fp32_oracle(orc, n, tile, ov, launch_per_cycle):
    h = 1.0 / (n + 1)
    f, x0 = W.rhs_random(n, n + tile), W.rhs_random(n, n + tile + 1)
    for s, nc in ((1, 3), (5, 4), (16, 2)):
        X = dev(x0)
        hj.solve_1d(dev(f), X, h, tile=tile, s=s, overlap=ov, rel_tol=0.0, max_cycles=nc,
                    launch_per_cycle=launch_per_cycle)
        assert np.array_equal(host32(X), orc.hier_1d_f32(f, x0, h, tile, s, nc, ov)), (n, tile, ov, s)


def test_fp32_batch_equals_fp32_oracle(orc):
    """FP32 problems of one batch (2D squares and rectangles, one with
    hx != hy, and 1D), fixed cycles, each equal to its FP32 oracle cycle."""
    specs = [((64, 64), 1.0 / 65, 1.0 / 65), ((70, 97), 1.0 / 98, 1.0 / 71), ((128, 150), 1.0 / 151, 1.0 / 151)]
    table, wants = [], []
    for k, ((ny, nx), hx, hy) in enumerate(specs):
        f = W.rhs_2d_modes(nx, ny, 8, 0.0, 40 + k)
        X = torch.zeros((ny, nx), dtype=F32, device="cuda")
        table.append((dev(f), X, hx, hy))
        wants.append(orc.hier_2d_f32(f, np.zeros((ny, nx)), hx, hy, (64, 64), 10, 7, (18, 18)))
    for k, n in enumerate((1000, 4000)):
        f = W.rhs_1d_modes(n, 8, 50 + k)
        X = torch.zeros(n, dtype=F32, device="cuda")
        table.append((dev(f), X, 1.0 / (n + 1), 1.0 / (n + 1)))
        wants.append(orc.hier_1d_f32(f, np.zeros(n), 1.0 / (n + 1), 256, 16, 7, 30))
    infos = hj.solve_batched(table, tile=(64, 64), s=10, overlap=(18, 18), tile_1d=256, s_1d=16, overlap_1d=30,
                             rel_tol=0.0, max_cycles=7, graph_cycles=3)
    for i, ((_, X, _, _), want) in enumerate(zip(table, wants)):
        assert infos[i].cycles == 7
        assert np.array_equal(host32(X), want), f"problem {i}"


@pytest.mark.parametrize("seed", [0, 5])
def test_refined_solve_is_oracle_fp64_cycles_plus_fp32_correction(orc, seed):
    """One refinement step rebuilt from the oracle, bit for bit: FP64 cycles
    up to the hand-over (fp64_cycles of them), r = f - A x in FP64 rounded to
    FP32, FP32 cycles on A e = r from e = 0 (inner_cycles of them), then
    x + e in FP64.  256^2, 64 x 32 tiles, s = 8, overlap 14, to 1e-10 with
    the hand-over allowed from the first cycle on."""
    n = 256
    h = 1.0 / (n + 1)
    kw = dict(tile=(64, 32), s=8, overlap=(14, 14))
    f = W.rhs_2d_modes(n, n, 8, 0.0, seed)
    X = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    info = hj.solve_2d_refined(torch.as_tensor(f).cuda(), X, h, rel_tol=1e-10, inner_tol=1e-6, switch_min_cycles=1,
                               **kw)
    say(f"refined seed {seed}: outer {info.outer}, fp64 {info.fp64_cycles}, fp32 {info.inner_cycles}")
    assert info.outer == 1 and info.inner_cycles > 0
    x1 = orc.hier_2d(f, np.zeros_like(f), h, h, kw["tile"], kw["s"], info.fp64_cycles, kw["overlap"])
    r, _ = orc.residual_2d(f, x1, h, h)
    e = orc.hier_2d_f32(r.astype(np.float32), np.zeros((n, n)), h, h, kw["tile"], kw["s"], info.inner_cycles,
                        kw["overlap"])
    want = x1 + e.astype(np.float64)
    torch.cuda.synchronize()
    assert np.array_equal(X.cpu().numpy(), want)
