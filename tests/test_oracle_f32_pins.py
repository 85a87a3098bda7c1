"""Pins of the oracle's FP32 sweeps and cycles (orc_*_f32), which check an
FP32 instantiation of the method bit for bit.

1. Where every operation is exact in single precision, FP32 and FP64 give the
   same numbers.  With h = 1 (so h^2 f = f) and small integer f and x0, an
   isotropic 2D update (h^2 f + S) / 4 stays a multiple of 4^-k of modest
   size for k sweeps, a 1D update one of 2^-k: exact in float for the few
   sweeps used here.  The FP32 cycle must then equal the FP64 oracle's cycle
   exactly, which pins everything but the rounding: tiles, halo, ownership,
   container parity, association (Sec. 3.3, 3.5, 4.1, 4.3).
2. In general the two differ by rounding only.  Each update rounds a handful
   of times (relative error u = 2^-24 each) and a Jacobi sweep does not grow
   an error in the max norm (its weights are non-negative and sum to at most
   1), so after K sweeps the FP32 result is within about
   K * c * u * (max |x| + max |h^2 f|) of the FP64 one; c = 8 covers the
   roundings of an update and of the coefficients.  A structural mistake in
   either code shows as an O(|x|) difference.
"""
import numpy as np
import pytest

from paper_2006_16465_amd import workloads as W

U = 2.0 ** -24


def ints(shape, seed):
    return np.random.default_rng(seed).integers(-16, 17, size=shape).astype(np.float64)


@pytest.mark.parametrize("tile,ov,s,nc", [((16, 16), (0, 0), 1, 3), ((16, 32), (6, 6), 3, 2), ((32, 16), (4, 2), 2, 3),
                                         ((8, 8), (2, 4), 6, 1), ((64, 16), (10, 0), 2, 2)])
def test_f32_cycle_2d_equals_f64_when_exact(orc, tile, ov, s, nc):
    f, x0 = ints((37, 53), 1), ints((37, 53), 2)
    a = orc.hier_2d(f, x0, 1.0, 1.0, tile, s, nc, ov)
    b = orc.hier_2d_f32(f, x0, 1.0, 1.0, tile, s, nc, ov)
    assert b.dtype == np.float32
    assert np.array_equal(a, b.astype(np.float64))


@pytest.mark.parametrize("tile,ov,s,nc", [(32, 0, 4, 3), (16, 6, 5, 2), (64, 14, 8, 2), (7, 2, 3, 4)])
def test_f32_cycle_1d_equals_f64_when_exact(orc, tile, ov, s, nc):
    f, x0 = ints(300, 3), ints(300, 4)
    a = orc.hier_1d(f, x0, 1.0, tile, s, nc, ov)
    b = orc.hier_1d_f32(f, x0, 1.0, tile, s, nc, ov)
    assert np.array_equal(a, b.astype(np.float64))


def test_f32_classical_equals_f64_when_exact(orc):
    f, x0 = ints((37, 53), 5), ints((37, 53), 6)
    assert np.array_equal(orc.jacobi_2d(f, x0, 1.0, 1.0, 6), orc.jacobi_2d_f32(f, x0, 1.0, 1.0, 6).astype(np.float64))
    f1, x1 = ints(300, 7), ints(300, 8)
    assert np.array_equal(orc.jacobi_1d(f1, x1, 1.0, 16), orc.jacobi_1d_f32(f1, x1, 1.0, 16).astype(np.float64))


def bound(K, *arrays):
    return 8.0 * U * K * sum(float(np.max(np.abs(a))) for a in arrays)


@pytest.mark.parametrize("hy_scale", [1.0, 1.7])
def test_f32_cycle_2d_within_rounding_of_f64(orc, hy_scale):
    ny, nx = 150, 200
    hx = 1.0 / (nx + 1)
    hy = hx * hy_scale
    f = W.rhs_2d_modes(nx, ny, 8, 0.1, 9)
    x0 = W.rhs_random((ny, nx), 10) * 1e-3
    # the FP32 code sees f and x0 rounded to float: compare from the same data
    f32, x32 = f.astype(np.float32).astype(np.float64), x0.astype(np.float32).astype(np.float64)
    tile, ov, s, nc = (32, 64), (14, 14), 8, 6
    a = orc.hier_2d(f32, x32, hx, hy, tile, s, nc, ov)
    b = orc.hier_2d_f32(f32, x32, hx, hy, tile, s, nc, ov).astype(np.float64)
    # the h^2 f term of an update, isotropic or not (f * dinv)
    hf = f32 * (hx * hx if hy_scale == 1.0 else 1.0 / (2.0 / hx ** 2 + 2.0 / hy ** 2))
    err = float(np.max(np.abs(a - b)))
    lim = bound(s * nc, a, x32, hf)
    assert 0.0 < err <= lim, (err, lim)


def test_f32_cycle_1d_within_rounding_of_f64(orc):
    n = 1000
    h = 1.0 / (n + 1)
    f = W.rhs_1d_modes(n, 8, 11).astype(np.float32).astype(np.float64)
    x0 = np.zeros(n)
    a = orc.hier_1d(f, x0, h, 64, 16, 10, 30)
    b = orc.hier_1d_f32(f, x0, h, 64, 16, 10, 30).astype(np.float64)
    err = float(np.max(np.abs(a - b)))
    assert 0.0 < err <= bound(160, a, f * h * h), err
