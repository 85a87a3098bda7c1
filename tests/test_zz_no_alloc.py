"""The allocation-free 2D solve (hj_solve_2d_noalloc) called through the C ABI
against hj_solve_2d on the same inputs: identical iterates, cycle counts and
residuals, on consecutive calls that reuse the one static scratch array (the
second smaller than the first, so stale contents of the larger call sit in
the scratch), and no device memory taken by the call itself."""
import ctypes

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def _call(name, F, X, h, p):
    """One solve through the C ABI; returns (status, info)."""
    ny, nx = F.shape
    info = hj._Info()
    fn = getattr(hj.load(), name)
    st = fn(nx, ny, F.stride(0), h, h, hj._dtype_code(F), F.data_ptr(), X.data_ptr(), ctypes.byref(p),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(info))
    torch.cuda.synchronize()
    return st, info


CASES = [
    # (ny, nx, dtype, tile, s, overlap, rel_tol, max_cycles, method)
    (768, 1024, torch.float64, (64, 64), 10, (18, 18), 1e-6, 100_000, "hierarchical"),
    (150, 200, torch.float64, (32, 32), 8, (0, 0), 0.0, 7, "hierarchical"),
    (120, 90, torch.float32, (64, 32), 6, (10, 10), 1e-4, 100_000, "hierarchical"),
    (64, 80, torch.float64, (32, 32), 1, (0, 0), 1e-3, 100_000, "global"),
]


def test_noalloc_equals_solve_2d_on_consecutive_calls():
    assert torch.cuda.is_available()
    for i, (ny, nx, dt, tile, s, ov, tol, mc, method) in enumerate(CASES):
        f = W.rhs_2d_modes(nx, ny, 8, 0.05, 20 + i)
        h = 1.0 / (nx + 1)
        p = hj.make_params(tile, s, method, tol, mc, 0, ov)
        F = _dev(f, dt)
        X1 = torch.zeros_like(F)
        X2 = torch.zeros_like(F)
        st1, i1 = _call("hj_solve_2d", F, X1, h, p)
        st2, i2 = _call("hj_solve_2d_noalloc", F, X2, h, p)
        print(f"case {i}: {ny}x{nx} {dt} tile {tile} s {s} ov {ov} tol {tol}: status {st1}/{st2}, "
              f"cycles {i1.cycles}/{i2.cycles}", flush=True)
        assert st1 == hj.HJ_OK and st2 == hj.HJ_OK, hj.last_error()
        assert torch.equal(X1, X2), f"case {i}: iterates differ"
        assert (i1.cycles, i1.sweeps) == (i2.cycles, i2.sweeps)
        assert i1.rel_residual == i2.rel_residual and i1.r0_norm == i2.r0_norm
        if tol > 0:
            assert i2.rel_residual <= tol


def test_noalloc_takes_no_device_memory():
    f = W.rhs_2d_modes(256, 256, 8, 0.0, 3)
    p = hj.make_params((64, 64), 10, "hierarchical", 1e-6, 100_000, 0, (18, 18))
    F = _dev(f, torch.float64)
    X = torch.zeros_like(F)
    assert _call("hj_solve_2d_noalloc", F, X, 1 / 257, p)[0] == hj.HJ_OK  # first call loads the code object
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        X.zero_()
        assert _call("hj_solve_2d_noalloc", F, X, 1 / 257, p)[0] == hj.HJ_OK
    assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_rejects_grids_beyond_its_scratch():
    # 2048 x 2048 FP64 fits (two 32 MiB iterate arrays), 2048 x 4096 does not
    F = torch.zeros((2048, 4096), dtype=torch.float64, device="cuda")
    X = torch.full_like(F, 3.0)
    p = hj.make_params((64, 64), 10, "hierarchical", 0.0, 1, 0, (18, 18))
    st, _ = _call("hj_solve_2d_noalloc", F, X, 1 / 4097, p)
    assert st == hj.HJ_ERR_INVALID_ARG and "bytes of scratch" in hj.last_error()
    assert bool((X == 3.0).all())
    G = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(G)
    st, info = _call("hj_solve_2d_noalloc", G, Y, 1 / 2049, p)
    assert st == hj.HJ_OK and info.cycles == 1
