"""ctypes binding of libhj.so (include/hj.h): argument marshalling only.

Every step of a solve runs in the HIP library; this module turns torch
tensors into device pointers, sizes and the current HIP stream, and turns
status codes into exceptions.  PyTorch supplies device memory and streams.

    import torch
    from paper_2006_16465_amd import hj
    f = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(f)
    info = hj.solve_2d(f, x, h=1 / 4097, tile=(32, 32), s=16, rel_tol=1e-6)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhj.so")

HJ_OK, HJ_ERR_INVALID_ARG, HJ_ERR_NOT_CONVERGED, HJ_ERR_NONFINITE, HJ_ERR_UNSUPPORTED, HJ_ERR_HIP = range(6)
HJ_F64, HJ_F32 = 0, 1
HJ_HIERARCHICAL, HJ_GLOBAL = 0, 1
HJ_FLAG_LDS_KERNEL = 0x1
HJ_FLAG_LAUNCH_PER_CYCLE = 0x2
METHODS = {"hierarchical": HJ_HIERARCHICAL, "global": HJ_GLOBAL}


class Params(ctypes.Structure):
    _fields_ = [
        ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
        ("overlap_x", ctypes.c_int32), ("overlap_y", ctypes.c_int32),
        ("s", ctypes.c_int32), ("method", ctypes.c_int32),
        ("max_cycles", ctypes.c_int64), ("check_every", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("rel_tol", ctypes.c_double),
    ]


class RefineParams(ctypes.Structure):
    _fields_ = [("inner", Params), ("rel_tol", ctypes.c_double), ("switch_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("switch_min_cycles", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _RefineInfo(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int64), ("inner_cycles", ctypes.c_int64),
                ("fp64_cycles", ctypes.c_int64), ("rel_residual", ctypes.c_double),
                ("r0_norm", ctypes.c_double)]


@dataclass
class RefineInfo:
    status: int
    outer: int
    inner_cycles: int
    fp64_cycles: int
    rel_residual: float
    r0_norm: float


class VCProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("a", ctypes.c_void_p), ("batch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("batch_stride", ctypes.c_int64)]


class AdjointDesc(ctypes.Structure):
    _fields_ = [("prob", VCProblem), ("u", ctypes.c_void_p), ("dl_du", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("dl_da", ctypes.c_void_p), ("ld_grad", ctypes.c_int64),
                ("params", Params)]


class TuneParams(ctypes.Structure):
    _fields_ = [("trial_tol", ctypes.c_double), ("max_trial_cycles", ctypes.c_int64),
                ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("rhs_stride", ctypes.c_int64)]


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("flags", ctypes.c_int32), ("nx", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("ld", ctypes.c_int64), ("hx", ctypes.c_double),
                ("hy", ctypes.c_double), ("f", ctypes.c_void_p), ("x", ctypes.c_void_p)]


class BatchParams(ctypes.Structure):
    _fields_ = [("p2", Params), ("p1", Params), ("rel_tol", ctypes.c_double),
                ("max_cycles", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("graph_cycles", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("max_outer", ctypes.c_int32)]


HJ_BATCH_AUTOTUNE = 0x1
HJ_BATCH_REFINE = 0x2
HJ_BATCH_WG1D = 0x4


class _Info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("rel_residual", ctypes.c_double), ("r0_norm", ctypes.c_double)]


@dataclass
class Info:
    status: int
    cycles: int
    sweeps: int
    rel_residual: float
    r0_norm: float

    @property
    def converged(self) -> bool:
        return self.status == HJ_OK


class HJError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_status_name(status)}: {detail}")
        self.status = status


_lib = None
EXPORTS = ("hj_params_default", "hj_solve_1d", "hj_solve_2d", "hj_solve_2d_noalloc", "hj_solve_2d_refined",
           "hj_residual",
           "hj_solve_batched", "hj_autotune", "hj_autotune_batch", "hj_autotune_solve", "hj_solve_vc_2d", "hj_vc_grad_a", "hj_solve_adjoint",
           "hj_axis_tiles",
           "hj_status_string", "hj_last_error", "hj_version")


def load():
    """Load libhj.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2006_16465_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, f64, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    P, I = ctypes.POINTER(Params), ctypes.POINTER(_Info)
    lib.hj_params_default.argtypes = [P]
    lib.hj_params_default.restype = None
    lib.hj_solve_1d.argtypes = [i64, f64, i32, vp, vp, P, vp, I]
    lib.hj_solve_1d.restype = i32
    lib.hj_solve_2d.argtypes = [i64, i64, i64, f64, f64, i32, vp, vp, P, vp, I]
    lib.hj_solve_2d.restype = i32
    lib.hj_solve_2d_noalloc.argtypes = [i64, i64, i64, f64, f64, i32, vp, vp, P, vp, I]
    lib.hj_solve_2d_noalloc.restype = i32
    lib.hj_solve_2d_refined.argtypes = [i64, i64, i64, f64, f64, vp, vp, ctypes.POINTER(RefineParams),
                                        vp, ctypes.POINTER(_RefineInfo)]
    lib.hj_solve_2d_refined.restype = i32
    lib.hj_residual.argtypes = [i32, i64, i64, i64, f64, f64, i32, vp, vp, vp, ctypes.POINTER(f64), vp]
    lib.hj_residual.restype = i32
    lib.hj_solve_batched.argtypes = [ctypes.POINTER(Problem), i64, ctypes.POINTER(BatchParams), vp, I]
    lib.hj_solve_batched.restype = i32
    lib.hj_autotune.argtypes = [i32, i64, i64, i32, vp, P, ctypes.POINTER(f64)]
    lib.hj_autotune.restype = i32
    lib.hj_autotune_batch.argtypes = [ctypes.POINTER(Problem), i64, i32, vp, P, P]
    lib.hj_autotune_batch.restype = i32
    lib.hj_autotune_solve.argtypes = [i64, i64, i64, f64, f64, i32, vp, vp, ctypes.POINTER(TuneParams), vp, P,
                                      ctypes.POINTER(f64)]
    lib.hj_autotune_solve.restype = i32
    lib.hj_solve_vc_2d.argtypes = [ctypes.POINTER(VCProblem), vp, vp, P, vp, I]
    lib.hj_solve_vc_2d.restype = i32
    lib.hj_vc_grad_a.argtypes = [ctypes.POINTER(VCProblem), vp, vp, vp, i64, vp]
    lib.hj_vc_grad_a.restype = i32
    lib.hj_solve_adjoint.argtypes = [ctypes.POINTER(AdjointDesc), vp, I]
    lib.hj_solve_adjoint.restype = i32
    lib.hj_axis_tiles.argtypes = [i64, i32, i32]
    lib.hj_axis_tiles.restype = i64
    lib.hj_status_string.argtypes = [i32]
    lib.hj_status_string.restype = ctypes.c_char_p
    lib.hj_last_error.argtypes = []
    lib.hj_last_error.restype = ctypes.c_char_p
    lib.hj_version.argtypes = []
    lib.hj_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    try:
        return load().hj_status_string(s).decode()
    except Exception:
        return f"status {s}"


def last_error() -> str:
    return load().hj_last_error().decode()


def axis_tiles(n: int, tile: int, overlap: int = 0) -> int:
    return int(load().hj_axis_tiles(n, tile, overlap))


def make_params(tile=32, s=16, method="hierarchical", rel_tol=1e-6, max_cycles=1_000_000,
                check_every=0, overlap=0, lds_kernel=False, launch_per_cycle=False) -> Params:
    p = Params()
    load().hj_params_default(ctypes.byref(p))
    tx, ty = (tile, tile) if isinstance(tile, int) else tile
    ox, oy = (overlap, overlap) if isinstance(overlap, int) else overlap
    p.tile_x, p.tile_y, p.overlap_x, p.overlap_y = tx, ty, ox, oy
    p.s = s
    p.method = METHODS[method] if isinstance(method, str) else int(method)
    p.rel_tol = rel_tol
    p.max_cycles = max_cycles
    p.check_every = check_every
    p.flags = (HJ_FLAG_LDS_KERNEL if lds_kernel else 0) | (HJ_FLAG_LAUNCH_PER_CYCLE if launch_per_cycle else 0)
    return p


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return HJ_F64
    if t.dtype == torch.float32:
        return HJ_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_pair(f, x):
    if not (f.is_cuda and x.is_cuda):
        raise ValueError("f and x must be GPU tensors")
    if f.dtype != x.dtype or f.shape != x.shape:
        raise ValueError("f and x must share dtype and shape")


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("2D tensors must be row-major with unit column stride")
    return t.stride(0)


def _raise_or_info(st: int, info: _Info, allow_not_converged: bool) -> Info:
    out = Info(st, info.cycles, info.sweeps, info.rel_residual, info.r0_norm)
    if st == HJ_OK or (st == HJ_ERR_NOT_CONVERGED and allow_not_converged):
        return out
    raise HJError(st, last_error())


def solve_1d(f, x, h, *, tile=32, s=16, method="hierarchical", rel_tol=1e-6, max_cycles=1_000_000,
             check_every=0, overlap=0, allow_not_converged=False, launch_per_cycle=False) -> Info:
    """Solve -u'' = f (n interior points, spacing h) in place in x (hj_solve_1d).
    Small hierarchical solves (tiles of 64-512 points, at most 16 tiles, f and
    two iterates within 150 KiB of LDS) run all their cycles in one workgroup;
    launch_per_cycle=True forces one kernel launch per cycle (same iterates)."""
    _check_pair(f, x)
    if f.dim() != 1 or not f.is_contiguous() or not x.is_contiguous():
        raise ValueError("1D tensors must be contiguous vectors")
    p = make_params(tile, s, method, rel_tol, max_cycles, check_every, overlap,
                    launch_per_cycle=launch_per_cycle)
    info = _Info()
    with _device(f):
        st = load().hj_solve_1d(f.numel(), float(h), _dtype_code(f), f.data_ptr(), x.data_ptr(),
                                ctypes.byref(p), _stream(f), ctypes.byref(info))
    return _raise_or_info(st, info, allow_not_converged)


def solve_2d(f, x, h=None, *, hx=None, hy=None, tile=(32, 32), s=16, method="hierarchical",
             rel_tol=1e-6, max_cycles=1_000_000, check_every=0, overlap=(0, 0),
             allow_not_converged=False, lds_kernel=False) -> Info:
    """Solve the 5-point Poisson system in place in x, f and x of shape (ny, nx) (hj_solve_2d).
    lds_kernel=True forces the LDS ping-pong cycle kernel (same iterates)."""
    _check_pair(f, x)
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    ld = _ld(f)
    if _ld(x) != ld:
        raise ValueError("f and x must share the row stride")
    ny, nx = f.shape
    p = make_params(tile, s, method, rel_tol, max_cycles, check_every, overlap, lds_kernel)
    info = _Info()
    with _device(f):
        st = load().hj_solve_2d(nx, ny, ld, float(hx), float(hy), _dtype_code(f), f.data_ptr(),
                                x.data_ptr(), ctypes.byref(p), _stream(f), ctypes.byref(info))
    return _raise_or_info(st, info, allow_not_converged)


NOALLOC_SCRATCH_BYTES = 96 << 20  # HJ_NOALLOC_SCRATCH_BYTES


def solve_2d_noalloc(f, x, h=None, *, hx=None, hy=None, tile=(32, 32), s=16, method="hierarchical",
                     rel_tol=1e-6, max_cycles=1_000_000, check_every=0, overlap=(0, 0),
                     allow_not_converged=False, lds_kernel=False) -> Info:
    """solve_2d without any allocation inside the library (hj_solve_2d_noalloc):
    its scratch is a fixed static device array of NOALLOC_SCRATCH_BYTES; larger
    grids raise HJError (HJ_ERR_INVALID_ARG).  Same iterates and info as solve_2d."""
    _check_pair(f, x)
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    ld = _ld(f)
    if _ld(x) != ld:
        raise ValueError("f and x must share the row stride")
    ny, nx = f.shape
    p = make_params(tile, s, method, rel_tol, max_cycles, check_every, overlap, lds_kernel)
    info = _Info()
    with _device(f):
        st = load().hj_solve_2d_noalloc(nx, ny, ld, float(hx), float(hy), _dtype_code(f), f.data_ptr(),
                                        x.data_ptr(), ctypes.byref(p), _stream(f), ctypes.byref(info))
    return _raise_or_info(st, info, allow_not_converged)


def solve_2d_refined(f, x, h=None, *, hx=None, hy=None, tile=(64, 32), s=8, overlap=(14, 14),
                     method="hierarchical", rel_tol=1e-10, inner_tol=1e-6, switch_tol=0.0,
                     inner_max_cycles=100_000, max_outer=50, check_every=0, switch_min_cycles=0,
                     allow_not_converged=False) -> RefineInfo:
    """FP64 solve: FP64 cycles down to switch_tol (0 = 1e4 * rel_tol, or
    1e5 * rel_tol when overlap >= 2s - 2 on both axes), then FP32 cycles inside
    FP64 iterative refinement (hj_solve_2d_refined); when the FP64 cycles
    reach switch_tol in fewer than switch_min_cycles (0 = 8) the solve stays
    FP64 to rel_tol (outer = 0).  f and x are FP64 (ny, nx) tensors; x is
    updated in place."""
    import torch
    _check_pair(f, x)
    if f.dtype != torch.float64:
        raise TypeError("solve_2d_refined takes FP64 f and x")
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    ld = _ld(f)
    if _ld(x) != ld:
        raise ValueError("f and x must share the row stride")
    ny, nx = f.shape
    rp = RefineParams()
    rp.inner = make_params(tile, s, method, inner_tol, inner_max_cycles, check_every, overlap)
    rp.rel_tol = rel_tol
    rp.switch_tol = switch_tol
    rp.max_outer = max_outer
    rp.flags = 0
    rp.switch_min_cycles = switch_min_cycles
    info = _RefineInfo()
    with _device(f):
        st = load().hj_solve_2d_refined(nx, ny, ld, float(hx), float(hy), f.data_ptr(), x.data_ptr(),
                                        ctypes.byref(rp), _stream(f), ctypes.byref(info))
    out = RefineInfo(st, info.outer, info.inner_cycles, info.fp64_cycles, info.rel_residual,
                     info.r0_norm)
    if st == HJ_OK or (st == HJ_ERR_NOT_CONVERGED and allow_not_converged):
        return out
    raise HJError(st, last_error())


def _problem_table(problems):
    """ctypes array of Problem for (f, x, h) / (f, x, hx, hy) entries, and the dtype code."""
    arr = (Problem * len(problems))()
    dt = None
    for i, pr in enumerate(problems):
        f, x = pr[0], pr[1]
        hx = float(pr[2])
        hy = float(pr[3]) if len(pr) > 3 else hx
        _check_pair(f, x)
        code = _dtype_code(f)
        if dt is None:
            dt = code
        elif code != dt:
            raise ValueError("all problems of a batch share one dtype")
        q = arr[i]
        q.flags = 0
        q.hx, q.hy = hx, hy
        q.f, q.x = f.data_ptr(), x.data_ptr()
        if f.dim() == 1:
            if not (f.is_contiguous() and x.is_contiguous()):
                raise ValueError("1D tensors must be contiguous")
            q.dim, q.nx, q.ny, q.ld = 1, f.numel(), 1, f.numel()
        elif f.dim() == 2:
            ld = _ld(f)
            if _ld(x) != ld:
                raise ValueError("f and x must share the row stride")
            q.dim, q.ny, q.nx, q.ld = 2, f.shape[0], f.shape[1], ld
        else:
            raise ValueError("problems are 1D or 2D tensors")
    return arr, dt


def autotune_batch(problems):
    """Cycle shapes hj_solve_batched(autotune=True) would use for this table:
    ((tile, s, overlap) for 2D, (tile, s, overlap) for 1D)."""
    arr, dt = _problem_table(problems)
    p2, p1 = Params(), Params()
    f0 = problems[0][0]
    with _device(f0):
        st = load().hj_autotune_batch(arr, len(problems), dt, _stream(f0), ctypes.byref(p2), ctypes.byref(p1))
    if st != HJ_OK:
        raise HJError(st, last_error())
    return ((p2.tile_x, p2.tile_y), p2.s, (p2.overlap_x, p2.overlap_y)), (p1.tile_x, p1.s, p1.overlap_x)


def solve_batched(problems, *, rel_tol=1e-8, tile=(64, 64), s=10, overlap=(18, 18), tile_1d=256,
                  s_1d=16, overlap_1d=30, max_cycles=1_000_000, graph_cycles=8, autotune=False,
                  refine=False, max_outer=0, allow_not_converged=False, one_workgroup_1d=False) -> list:
    """Solve many independent problems together (hj_solve_batched).

    problems: sequence of (f, x, h) or (f, x, hx, hy); f, x GPU tensors of one
    dtype, shape (n,) for 1D and (ny, nx) for 2D (row-major).  Each x is updated
    in place.  2D problems use the cycle (tile, s, overlap), 1D problems
    (tile_1d, s_1d, overlap_1d); autotune=True lets the library choose both.
    refine=True (FP64 problems): each problem on its own schedule, FP64 cycles
    down to min(1e4 rel_tol, rel_tol / 8F) (F its FP32 floor predicted from its
    measured convergence rate), then FP32 correction cycles inside FP64
    refinement (at most max_outer correction solves, 0 = 8; a problem whose
    FP32 solve stops converging, or whose F is too large, continues in FP64).
    max_cycles bounds every problem's cycles over all phases.  Info.cycles
    counts the cycles inside each result.  one_workgroup_1d=True (1D problems
    only, tile_1d of 64-512, at most 16 tiles and 150 KiB of f and iterates per
    problem): each problem runs its whole solve inside one workgroup, one
    launch for the batch.  Returns one Info per problem."""
    import torch
    if not problems:
        return []
    arr, dt = _problem_table(problems)
    bp = BatchParams()
    bp.p2 = make_params(tile, s, "hierarchical", rel_tol, max_cycles, 0, overlap)
    bp.p1 = make_params(tile_1d, s_1d, "hierarchical", rel_tol, max_cycles, 0, overlap_1d)
    bp.rel_tol = rel_tol
    bp.max_cycles = max_cycles
    bp.dtype = dt
    bp.graph_cycles = graph_cycles
    bp.flags = ((HJ_BATCH_AUTOTUNE if autotune else 0) | (HJ_BATCH_REFINE if refine else 0) |
                (HJ_BATCH_WG1D if one_workgroup_1d else 0))
    bp.max_outer = max_outer
    infos = (_Info * len(problems))()
    f0 = problems[0][0]
    with _device(f0):
        st = load().hj_solve_batched(arr, len(problems), ctypes.byref(bp), _stream(f0), infos)
    if st != HJ_OK and not (st == HJ_ERR_NOT_CONVERGED and allow_not_converged):
        raise HJError(st, last_error())
    out = []
    for i in infos:
        # per problem, as the device judged it: met rel_tol, went non-finite, or ran out of cycles
        if i.rel_residual != i.rel_residual:
            ps = HJ_ERR_NONFINITE
        elif rel_tol > 0.0 and i.rel_residual > rel_tol:
            ps = HJ_ERR_NOT_CONVERGED
        else:
            ps = HJ_OK
        out.append(Info(ps, i.cycles, i.sweeps, i.rel_residual, i.r0_norm))
    return out


def autotune_solve(f, x0=None, h=None, *, hx=None, hy=None, trial_tol=1e-6, max_trial_cycles=1_000_000,
                   tile=None):
    """Cycle shape that solves this 2D problem (f, from x0, default 0) to
    trial_tol fastest, inexact overlaps included (hj_autotune_solve).
    f may be (nrhs, ny, nx), contiguous: several right-hand sides, scored by
    the sum of their trial times (every one must reach trial_tol); x0 is
    (ny, nx) and shared.  tile=(tx, ty) restricts the candidates to that
    tile.  Returns (tile, s, overlap, ms of the winning trials)."""
    import torch
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    nrhs = 0
    if f.dim() == 3:
        if not f.is_contiguous():
            raise ValueError("a stack of right-hand sides must be contiguous")
        nrhs = f.shape[0]
        f2 = f[0]
    else:
        f2 = f
    x0 = torch.zeros_like(f2) if x0 is None else x0
    _check_pair(f2, x0)
    ld = _ld(f2)
    if _ld(x0) != ld:
        raise ValueError("f and x0 must share the row stride")
    ny, nx = f2.shape
    tp = TuneParams()
    tp.trial_tol, tp.max_trial_cycles, tp.flags = trial_tol, max_trial_cycles, 0
    tp.tile_x, tp.tile_y = tile if tile is not None else (0, 0)
    tp.nrhs, tp.rhs_stride = nrhs, (f.stride(0) if nrhs else 0)
    p = Params()
    ms = ctypes.c_double()
    with _device(f):
        st = load().hj_autotune_solve(nx, ny, ld, float(hx), float(hy), _dtype_code(f2), f.data_ptr(),
                                      x0.data_ptr(), ctypes.byref(tp), _stream(f), ctypes.byref(p), ctypes.byref(ms))
    if st != HJ_OK:
        raise HJError(st, last_error())
    return (p.tile_x, p.tile_y), p.s, (p.overlap_x, p.overlap_y), ms.value


def autotune(dim, nx, ny=1, dtype=None):
    """Fastest cycle shape per sweep for an nx x ny (1D: nx) grid (hj_autotune).
    Returns (tile, s, overlap, microseconds per sweep); tile and overlap are
    (x, y) pairs in 2D and ints in 1D."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    code = HJ_F64 if dtype == torch.float64 else HJ_F32
    p = Params()
    us = ctypes.c_double()
    st = load().hj_autotune(dim, nx, ny, code, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                            ctypes.byref(p), ctypes.byref(us))
    if st != HJ_OK:
        raise HJError(st, last_error())
    if dim == 2:
        return (p.tile_x, p.tile_y), p.s, (p.overlap_x, p.overlap_y), us.value
    return p.tile_x, p.s, p.overlap_x, us.value


def _vc_problem(a, f, hx, hy):
    """f: (ny, nx) or (batch, ny, nx) contiguous FP64; a: (ny+2, nx+2) contiguous FP64."""
    import torch
    if f.dtype != torch.float64 or a.dtype != torch.float64:
        raise TypeError("variable-coefficient solves are FP64")
    if not (f.is_cuda and a.is_cuda and f.is_contiguous() and a.is_contiguous()):
        raise ValueError("a and f must be contiguous GPU tensors")
    ny, nx = f.shape[-2:]
    if tuple(a.shape) != (ny + 2, nx + 2):
        raise ValueError(f"a must have shape {(ny + 2, nx + 2)}")
    pr = VCProblem()
    pr.nx, pr.ny, pr.ld, pr.lda = nx, ny, nx, nx + 2
    pr.hx, pr.hy = float(hx), float(hy)
    pr.a = a.data_ptr()
    pr.batch = f.shape[0] if f.dim() == 3 else 1
    pr.flags = 0
    pr.batch_stride = ny * nx
    return pr


def solve_vc_2d(a, f, u, h=None, *, hx=None, hy=None, tile=(32, 32), s=8, overlap=(0, 0),
                method="hierarchical", rel_tol=1e-10, max_cycles=1_000_000, check_every=0,
                allow_not_converged=False, lds_kernel=False):
    """Solve -div(a grad u_b) = f_b for a batch (hj_solve_vc_2d); u (same shape as f) in/out.
    Returns one Info per right-hand side.  lds_kernel: HJ_FLAG_LDS_KERNEL."""
    _check_pair(f, u)
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    pr = _vc_problem(a, f, hx, hy)
    if not u.is_contiguous():
        raise ValueError("u must be contiguous")
    p = make_params(tile, s, method, rel_tol, max_cycles, check_every, overlap, lds_kernel=lds_kernel)
    infos = (_Info * pr.batch)()
    with _device(f):
        st = load().hj_solve_vc_2d(ctypes.byref(pr), f.data_ptr(), u.data_ptr(), ctypes.byref(p),
                                   _stream(f), infos)
    out = [Info(st, i.cycles, i.sweeps, i.rel_residual, i.r0_norm) for i in infos]
    if st == HJ_OK or (st == HJ_ERR_NOT_CONVERGED and allow_not_converged):
        return out
    raise HJError(st, last_error())


def vc_grad_a(a, u, lam, h=None, *, hx=None, hy=None):
    """dL/da (shape of a) from forward states u and adjoint states lam, summed over the batch."""
    import torch
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    pr = _vc_problem(a, u, hx, hy)
    if lam.shape != u.shape or not lam.is_contiguous():
        raise ValueError("lam must match u")
    grad = torch.empty_like(a)
    with _device(u):
        st = load().hj_vc_grad_a(ctypes.byref(pr), u.data_ptr(), lam.data_ptr(), grad.data_ptr(),
                                 a.shape[1], _stream(u))
    if st != HJ_OK:
        raise HJError(st, last_error())
    return grad


def solve_adjoint(a, u, dl_du, lam, h=None, *, hx=None, hy=None, tile=(32, 32), s=8, overlap=(0, 0),
                  method="hierarchical", rel_tol=1e-10, max_cycles=1_000_000, check_every=0, grad_a=True,
                  allow_not_converged=False):
    """Backward pass of the variable-coefficient solve (hj_solve_adjoint): solves
    A(a) lam_b = dL/du_b in place in lam (lam holds the initial guess on entry;
    A is symmetric, so this is the forward solve on dL/du), which is dL/df, and,
    with grad_a, dL/da from the forward states u and lam summed over the batch.
    u, dl_du, lam: (ny, nx) or (batch, ny, nx) contiguous FP64; a: (ny+2, nx+2).
    Returns (infos, dl_da or None)."""
    import torch
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    _check_pair(dl_du, lam)
    pr = _vc_problem(a, dl_du, hx, hy)
    if not lam.is_contiguous():
        raise ValueError("lam must be contiguous")
    if grad_a and (u.shape != dl_du.shape or u.dtype != dl_du.dtype or not u.is_cuda or not u.is_contiguous()):
        raise ValueError("u must match dl_du")
    d = AdjointDesc()
    d.prob = pr
    d.u = u.data_ptr() if grad_a else None
    d.dl_du = dl_du.data_ptr()
    d.lam = lam.data_ptr()
    grad = torch.empty_like(a) if grad_a else None
    d.dl_da = grad.data_ptr() if grad_a else None
    d.ld_grad = a.shape[1]
    d.params = make_params(tile, s, method, rel_tol, max_cycles, check_every, overlap)
    infos = (_Info * pr.batch)()
    with _device(dl_du):
        st = load().hj_solve_adjoint(ctypes.byref(d), _stream(dl_du), infos)
    out = [Info(st, i.cycles, i.sweeps, i.rel_residual, i.r0_norm) for i in infos]
    if st == HJ_OK or (st == HJ_ERR_NOT_CONVERGED and allow_not_converged):
        return out, grad
    raise HJError(st, last_error())


def _diffusion_fn():
    import torch

    class DiffusionSolve(torch.autograd.Function):
        """u = A(a)^-1 f for -div(a grad u) = f.  Backward: one call of
        hj_solve_adjoint -- the adjoint solve A lam = dL/du (A is symmetric),
        dL/df = lam, and dL/da from the face products of u and lam.  Only the
        converged u (and a) are stored."""

        @staticmethod
        def forward(ctx, f, a, opts):
            f = f.contiguous()
            a = a.contiguous()
            u = torch.zeros_like(f)
            solve_vc_2d(a, f, u, **opts)
            ctx.save_for_backward(u, a)
            ctx.opts = opts
            return u

        @staticmethod
        def backward(ctx, grad_u):
            u, a = ctx.saved_tensors
            g = grad_u.contiguous()
            lam = torch.zeros_like(g)
            _, grad_a = solve_adjoint(a, u, g, lam, grad_a=ctx.needs_input_grad[1], **ctx.opts)
            return lam, grad_a, None

    return DiffusionSolve


_DIFF = None


def diffusion_solve(f, a, h=None, *, hx=None, hy=None, tile=(32, 32), s=8, overlap=(0, 0),
                    rel_tol=1e-10, max_cycles=1_000_000):
    """Differentiable variable-coefficient solve (torch autograd): returns u with
    gradients to f and a through the adjoint hierarchical solve."""
    global _DIFF
    if _DIFF is None:
        _DIFF = _diffusion_fn()
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    opts = dict(hx=hx, hy=hy, tile=tile, s=s, overlap=overlap, rel_tol=rel_tol, max_cycles=max_cycles)
    return _DIFF.apply(f, a, opts)


def residual(f, x, h=None, *, hx=None, hy=None, r_out=None) -> float:
    """||f - A x||_2 (FP64); fills r_out with f - A x when given (hj_residual)."""
    _check_pair(f, x)
    hx = hx if hx is not None else h
    hy = hy if hy is not None else hx
    if r_out is not None and (r_out.dtype != f.dtype or r_out.shape != f.shape or not r_out.is_cuda):
        raise ValueError("r_out must match f")
    nrm = ctypes.c_double(0.0)
    rp = r_out.data_ptr() if r_out is not None else None
    with _device(f):
        if f.dim() == 1:
            st = load().hj_residual(1, f.numel(), 1, f.numel(), float(hx), float(hx), _dtype_code(f),
                                    f.data_ptr(), x.data_ptr(), rp, ctypes.byref(nrm), _stream(f))
        else:
            ld = _ld(f)
            if _ld(x) != ld or (r_out is not None and _ld(r_out) != ld):
                raise ValueError("f, x and r_out must share the row stride")
            ny, nx = f.shape
            st = load().hj_residual(2, nx, ny, ld, float(hx), float(hy), _dtype_code(f),
                                    f.data_ptr(), x.data_ptr(), rp, ctypes.byref(nrm), _stream(f))
    if st != HJ_OK:
        raise HJError(st, last_error())
    return nrm.value


class _device:
    """Make the tensor's GPU current for the duration of a library call."""

    def __init__(self, t):
        self.idx = t.device.index

    def __enter__(self):
        import torch
        self.prev = torch.cuda.current_device()
        if self.idx is not None and self.idx != self.prev:
            torch.cuda.set_device(self.idx)

    def __exit__(self, *a):
        import torch
        if self.idx is not None and self.idx != self.prev:
            torch.cuda.set_device(self.prev)
