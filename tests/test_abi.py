"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/hj.h declares, and rejects invalid arguments before touching
the HIP runtime."""
import ctypes
import os
import re

import pytest

from paper_2006_16465_amd import hj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hj.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hj_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hj_solve_1d", "hj_solve_2d", "hj_solve_2d_refined", "hj_residual", "hj_solve_batched",
              "hj_solve_vc_2d", "hj_vc_grad_a", "hj_solve_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = hj.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(hj.EXPORTS) == set(declared_functions())


def _params(**kw):
    p = hj.Params()
    hj.load().hj_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


FAKE = 0x10000  # aligned non-NULL pointer; validation must reject before it is used


@pytest.mark.parametrize("args,kw,code", [
    ((0, 8, 8, 0.1, 0.1, 0), {}, hj.HJ_ERR_INVALID_ARG),         # nx = 0
    ((8, 0, 8, 0.1, 0.1, 0), {}, hj.HJ_ERR_INVALID_ARG),         # ny = 0
    ((8, 8, 7, 0.1, 0.1, 0), {}, hj.HJ_ERR_INVALID_ARG),         # ld < nx
    ((8, 8, 8, 0.0, 0.1, 0), {}, hj.HJ_ERR_INVALID_ARG),         # hx = 0
    ((8, 8, 8, 0.1, float("nan"), 0), {}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 7), {}, hj.HJ_ERR_INVALID_ARG),         # dtype
    ((8, 8, 8, 0.1, 0.1, 0), {"s": 0}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"max_cycles": 0}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"overlap_x": 32}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"overlap_y": -2}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"method": 5}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"flags": 4}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"rel_tol": float("nan")}, hj.HJ_ERR_INVALID_ARG),
    ((8, 8, 8, 0.1, 0.1, 0), {"tile_x": 48}, hj.HJ_ERR_UNSUPPORTED),
    ((8, 8, 8, 0.1, 0.1, 0), {"tile_x": 16, "tile_y": 128}, hj.HJ_ERR_UNSUPPORTED),
    ((8, 8, 8, 0.1, 0.1, 0), {"tile_y": 256}, hj.HJ_ERR_UNSUPPORTED),
    # 128-extent tiles only on grids of at least one full tile, register kernel only
    ((100, 200, 100, 0.1, 0.1, 0), {"tile_x": 128, "tile_y": 64}, hj.HJ_ERR_UNSUPPORTED),
    ((200, 100, 200, 0.1, 0.1, 0), {"tile_x": 64, "tile_y": 128}, hj.HJ_ERR_UNSUPPORTED),
    ((256, 256, 256, 0.1, 0.1, 0), {"tile_x": 128, "tile_y": 128, "flags": 1}, hj.HJ_ERR_UNSUPPORTED),
])
@pytest.mark.parametrize("entry", ["hj_solve_2d", "hj_solve_2d_noalloc"])
def test_solve_2d_rejects_invalid_arguments(args, kw, code, entry):
    lib = hj.load()
    info = hj._Info()
    p = _params(**kw)
    st = getattr(lib, entry)(*args, FAKE, FAKE, ctypes.byref(p), None, ctypes.byref(info))
    assert st == code, hj.last_error()
    assert hj.last_error()


@pytest.mark.parametrize("nx,ny,ld,dtype", [(4096, 2048, 4096, hj.HJ_F64), (3072, 2048, 3072, hj.HJ_F64),
                                            (2048, 2048, 3100, hj.HJ_F64), (4096, 4096, 4096, hj.HJ_F32)])
def test_noalloc_rejects_grids_beyond_its_scratch_before_any_hip_call(nx, ny, ld, dtype):
    """Two iterate arrays of ny * ld elements plus the partials must fit the
    static scratch; larger grids fail up front (FAKE pointers are never used)."""
    lib = hj.load()
    info = hj._Info()
    p = _params(tile_x=64, tile_y=64, s=10, overlap_x=18, overlap_y=18)
    st = lib.hj_solve_2d_noalloc(nx, ny, ld, 0.01, 0.01, dtype, FAKE, FAKE, ctypes.byref(p), None,
                                 ctypes.byref(info))
    assert st == hj.HJ_ERR_INVALID_ARG
    assert "bytes of scratch" in hj.last_error() and str(hj.NOALLOC_SCRATCH_BYTES) in hj.last_error()


def test_solve_rejects_null_and_misaligned_pointers():
    lib = hj.load()
    info = hj._Info()
    p = _params()
    assert lib.hj_solve_2d(8, 8, 8, 0.1, 0.1, 0, None, FAKE, ctypes.byref(p), None, ctypes.byref(info)) == 1
    assert lib.hj_solve_2d(8, 8, 8, 0.1, 0.1, 0, FAKE + 4, FAKE, ctypes.byref(p), None, ctypes.byref(info)) == 1
    assert lib.hj_solve_2d(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, None, None, ctypes.byref(info)) == 1
    assert lib.hj_solve_1d(0, 0.1, 0, FAKE, FAKE, ctypes.byref(p), None, ctypes.byref(info)) == 1
    assert lib.hj_solve_1d(16, -1.0, 0, FAKE, FAKE, ctypes.byref(p), None, ctypes.byref(info)) == 1
    p1 = _params(tile_x=48)
    assert lib.hj_solve_1d(16, 0.1, 0, FAKE, FAKE, ctypes.byref(p1), None, ctypes.byref(info)) == hj.HJ_ERR_UNSUPPORTED
    # flags: HJ_FLAG_LAUNCH_PER_CYCLE passes validation (the call then needs a
    # device); an unknown bit does not
    pf = _params(tile_x=64, flags=hj.HJ_FLAG_LAUNCH_PER_CYCLE)
    assert lib.hj_solve_1d(16, 0.1, 0, FAKE, FAKE, ctypes.byref(pf), None, ctypes.byref(info)) != 1
    pf = _params(tile_x=64, flags=8)
    assert lib.hj_solve_1d(16, 0.1, 0, FAKE, FAKE, ctypes.byref(pf), None, ctypes.byref(info)) == 1
    nrm = ctypes.c_double()
    assert lib.hj_residual(3, 8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, None, ctypes.byref(nrm), None) == 1
    assert lib.hj_residual(2, 8, 8, 4, 0.1, 0.1, 0, FAKE, FAKE, None, ctypes.byref(nrm), None) == 1
    assert lib.hj_residual(2, 8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, FAKE + 2, ctypes.byref(nrm), None) == 1


def test_refined_solve_rejects_invalid_arguments():
    lib = hj.load()
    info = hj._RefineInfo()

    def rp(**kw):
        p = hj.RefineParams()
        p.inner = _params(rel_tol=1e-4)
        p.rel_tol, p.max_outer, p.flags = 1e-10, 10, 0
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    def call(p, nx=8, ny=8, ld=8, h=0.1):
        return lib.hj_solve_2d_refined(nx, ny, ld, h, h, FAKE, FAKE, ctypes.byref(p), None, ctypes.byref(info))

    assert call(rp(rel_tol=0.0)) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(max_outer=0)) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(flags=1)) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(switch_min_cycles=-1)) == hj.HJ_ERR_INVALID_ARG
    assert ctypes.sizeof(hj.RefineParams) == 80  # hj_refine_params in include/hj.h
    assert call(rp(switch_tol=-1e-3)) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(switch_tol=float("nan"))) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(switch_tol=float("inf"))) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(inner=_params(rel_tol=0.0))) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(inner=_params(rel_tol=1e-4, s=0))) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(inner=_params(rel_tol=1e-4, tile_x=48))) == hj.HJ_ERR_UNSUPPORTED
    assert call(rp(), ld=4) == hj.HJ_ERR_INVALID_ARG
    assert call(rp(), h=-1.0) == hj.HJ_ERR_INVALID_ARG


def _batch(n2=1, n1=1, **kw):
    arr = (hj.Problem * (n2 + n1))()
    for i in range(n2 + n1):
        q = arr[i]
        q.dim, q.flags = (2, 0) if i < n2 else (1, 0)
        q.nx, q.ny, q.ld = (300, 200, 300) if i < n2 else (5000, 1, 5000)
        q.hx = q.hy = 0.01
        q.f, q.x = FAKE, FAKE + 0x1000
    bp = hj.BatchParams()
    bp.p2 = _params(tile_x=64, tile_y=64, s=10, overlap_x=18, overlap_y=18)
    bp.p1 = _params(tile_x=256, s=16, overlap_x=30)
    bp.rel_tol, bp.max_cycles, bp.dtype, bp.graph_cycles, bp.flags = 1e-8, 100, 0, 8, 0
    for k, v in kw.items():
        if k.startswith("q_"):
            setattr(arr[0], k[2:], v)
        else:
            setattr(bp, k, v)
    return arr, bp


@pytest.mark.parametrize("kw,code", [
    ({"q_dim": 3}, hj.HJ_ERR_INVALID_ARG),
    ({"q_flags": 1}, hj.HJ_ERR_INVALID_ARG),
    ({"q_ld": 100}, hj.HJ_ERR_INVALID_ARG),             # ld < nx
    ({"q_hy": 0.0}, hj.HJ_ERR_INVALID_ARG),
    ({"q_hx": float("inf")}, hj.HJ_ERR_INVALID_ARG),
    ({"q_x": None}, hj.HJ_ERR_INVALID_ARG),
    ({"q_f": FAKE + 3}, hj.HJ_ERR_INVALID_ARG),         # misaligned
    ({"q_nx": 0}, hj.HJ_ERR_INVALID_ARG),
    ({"dtype": 7}, hj.HJ_ERR_INVALID_ARG),
    ({"max_cycles": 0}, hj.HJ_ERR_INVALID_ARG),
    ({"graph_cycles": 2000}, hj.HJ_ERR_INVALID_ARG),
    ({"flags": 8}, hj.HJ_ERR_INVALID_ARG),
    ({"flags": 6}, hj.HJ_ERR_UNSUPPORTED),              # HJ_BATCH_WG1D with HJ_BATCH_REFINE
    ({"rel_tol": float("nan")}, hj.HJ_ERR_INVALID_ARG),
    ({"q_nx": 40, "q_ld": 40}, hj.HJ_ERR_UNSUPPORTED),   # 2D problem smaller than the tile
])
def test_batched_rejects_invalid_arguments(kw, code):
    lib = hj.load()
    arr, bp = _batch(**kw)
    infos = (hj._Info * len(arr))()
    assert lib.hj_solve_batched(arr, len(arr), ctypes.byref(bp), None, infos) == code, hj.last_error()
    assert hj.last_error()


def test_batched_rejects_unsupported_shapes_and_empty_tables():
    lib = hj.load()
    arr, bp = _batch()
    assert lib.hj_solve_batched(None, 1, ctypes.byref(bp), None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_solve_batched(arr, 0, ctypes.byref(bp), None, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_solve_batched(arr, 2, None, None, None) == hj.HJ_ERR_INVALID_ARG
    for p2 in (_params(tile_x=128, tile_y=64), _params(tile_x=16, tile_y=16),
               _params(tile_x=64, tile_y=64, method=hj.HJ_GLOBAL)):
        arr, bp = _batch()
        bp.p2 = p2
        assert lib.hj_solve_batched(arr, 2, ctypes.byref(bp), None, None) == hj.HJ_ERR_UNSUPPORTED
    arr, bp = _batch()
    bp.p1 = _params(tile_x=48)
    assert lib.hj_solve_batched(arr, 2, ctypes.byref(bp), None, None) == hj.HJ_ERR_UNSUPPORTED


def test_autotune_validates():
    lib = hj.load()
    p = hj.Params()
    us = ctypes.c_double()
    assert lib.hj_autotune(3, 64, 64, 0, None, ctypes.byref(p), ctypes.byref(us)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_autotune(2, 0, 64, 0, None, ctypes.byref(p), ctypes.byref(us)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_autotune(2, 64, 64, 5, None, ctypes.byref(p), ctypes.byref(us)) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_autotune(1, 64, 1, 0, None, None, None) == hj.HJ_ERR_INVALID_ARG


def test_variable_coefficient_entry_points_validate():
    lib = hj.load()
    p = _params()

    def prob(**kw):
        pr = hj.VCProblem()
        pr.nx, pr.ny, pr.ld, pr.lda, pr.hx, pr.hy = 8, 8, 8, 10, 0.1, 0.1
        pr.a, pr.batch, pr.flags, pr.batch_stride = FAKE, 1, 0, 64
        for k, v in kw.items():
            setattr(pr, k, v)
        return pr

    info = (hj._Info * 4)()
    for kw in ({"nx": 0}, {"ld": 7}, {"lda": 9}, {"hx": 0.0}, {"batch": 0}, {"flags": 1},
               {"batch": 2, "batch_stride": 10}, {"a": None}):
        pr = prob(**kw)
        assert lib.hj_solve_vc_2d(ctypes.byref(pr), FAKE, FAKE, ctypes.byref(p), None, info) == \
            hj.HJ_ERR_INVALID_ARG, kw
    pr = prob()
    assert lib.hj_vc_grad_a(ctypes.byref(pr), FAKE, FAKE, FAKE, 9, None) == hj.HJ_ERR_INVALID_ARG
    assert lib.hj_solve_adjoint(None, None, None) == hj.HJ_ERR_INVALID_ARG
    # the adjoint descriptor is checked whole before its solve runs: a
    # requested gradient without forward states, a short gradient pitch, a
    # misaligned or missing pointer, or a bad problem all fail up front
    def desc(**kw):
        d = hj.AdjointDesc()
        d.prob = prob()
        d.u, d.dl_du, d.lam, d.dl_da, d.ld_grad = FAKE, FAKE, FAKE, FAKE, 10
        d.params = _params()
        for k, v in kw.items():
            setattr(d, k, v)
        return d
    for kw in ({"u": None}, {"ld_grad": 9}, {"dl_du": None}, {"lam": None}, {"lam": FAKE + 4},
               {"dl_da": FAKE + 2}, {"prob": prob(nx=0)}):
        d = desc(**kw)
        assert lib.hj_solve_adjoint(ctypes.byref(d), None, info) == hj.HJ_ERR_INVALID_ARG, kw
        assert hj.last_error(), kw


def test_status_strings_and_defaults():
    lib = hj.load()
    assert lib.hj_status_string(0) == b"HJ_OK"
    assert lib.hj_status_string(2) == b"HJ_ERR_NOT_CONVERGED"
    p = _params()
    assert (p.tile_x, p.tile_y, p.s, p.method, p.check_every) == (32, 32, 16, 0, 0)
    assert p.rel_tol == 1e-6 and p.flags == 0 and hj.HJ_FLAG_LDS_KERNEL == 1


@pytest.mark.parametrize("n,t,o", [(4096, 32, 0), (4096, 32, 4), (1000, 64, 6), (7, 32, 0), (12, 4, 2)])
def test_partition_count_agrees_with_oracle(orc, n, t, o):
    assert hj.axis_tiles(n, t, o) == len(orc.axis_tiles(n, t, o))
    assert hj.axis_tiles(0, 32, 0) == -1 and hj.axis_tiles(10, 8, 8) == -1


def test_autotune_solve_rejects_invalid_arguments():
    lib = hj.load()

    def tp(**kw):
        t = hj.TuneParams()
        t.trial_tol, t.max_trial_cycles, t.tile_x, t.tile_y, t.flags = 1e-4, 1000, 0, 0, 0
        for k, v in kw.items():
            setattr(t, k, v)
        return t

    best = hj.Params()
    ms = ctypes.c_double()

    def call(t, nx=64, ny=64, ld=64, x0=FAKE):
        return lib.hj_autotune_solve(nx, ny, ld, 0.01, 0.01, 0, FAKE, x0, ctypes.byref(t) if t else None, None,
                                     ctypes.byref(best), ctypes.byref(ms))

    assert call(None) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(trial_tol=0.0)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(trial_tol=float("nan"))) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(max_trial_cycles=0)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(flags=1)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(tile_x=64)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(tile_x=48, tile_y=32)) == hj.HJ_ERR_UNSUPPORTED
    assert call(tp(), ld=32) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(), x0=None) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(nrhs=-1)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(nrhs=1025, rhs_stride=64 * 64)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(nrhs=2, rhs_stride=64 * 64 - 1)) == hj.HJ_ERR_INVALID_ARG
    assert call(tp(nrhs=2, rhs_stride=-64)) == hj.HJ_ERR_INVALID_ARG
    # ny * ld overflows int64 here: the check must not wrap
    assert call(tp(nrhs=3, rhs_stride=1 << 62), ld=1 << 60) == hj.HJ_ERR_INVALID_ARG
    assert hj.last_error()
    assert ctypes.sizeof(hj.TuneParams) == 40

