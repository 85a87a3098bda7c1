"""CPU FP64 oracle for hierarchical Jacobi (test infrastructure only).

Thin ctypes wrapper over ``hj_oracle.c``.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark import this package; the product
library (``paper_2006_16465_amd``) never does, and the two share no code.

Every function takes and returns NumPy float64 arrays on the host.  1D arrays
hold the n interior points; 2D arrays are row-major ``[ny, nx]`` (row = y
index).  The paper's definitions followed by each function are cited in the C
source; briefly:

* ``jacobi_*``   classical Jacobi sweeps (Sec. 3.1, update eqs. of Sec. 3.4
  and Sec. 4.2);
* ``hier_*``     hierarchical cycles (Sec. 3.3 three-step cycle, Sec. 4.1 in
  2D, overlapping subdomains Sec. 3.5 / Sec. 4.3);
* ``residual_*`` r = f - A x and its 2-norm (stopping rule of Sec. 3.4);
* ``solve_*``    iterate until ||r_n|| <= tol ||r_0||, checking every cycle;
* ``*_f32``      the same sweeps and cycles in single precision, for checking
  an FP32 instantiation (float32 in and out).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhj_oracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f64 = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pf = ctypes.POINTER(ctypes.c_float)
_pi64 = ctypes.POINTER(ctypes.c_int64)

HIERARCHICAL = 0
CLASSICAL = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_axis_ntiles": (_i64, [_i64, _i64, _i64]),
        "orc_axis_start": (_i64, [_i64, _i64, _i64, _i64]),
        "orc_axis_owned": (None, [_i64, _i64, _i64, _i64, _pi64, _pi64]),
        "orc_jacobi_1d": (None, [_i64, _f64, _pd, _pd, _i64]),
        "orc_jacobi_2d": (None, [_i64, _i64, _f64, _f64, _pd, _pd, _i64]),
        "orc_hier_1d": (None, [_i64, _f64, _pd, _pd, _i64, _i64, _i64, _i64]),
        "orc_hier_2d": (None, [_i64, _i64, _f64, _f64, _pd, _pd, _i64, _i64, _i64, _i64, _i64, _i64]),
        "orc_jacobi_1d_f32": (None, [_i64, _f64, _pf, _pf, _i64]),
        "orc_jacobi_2d_f32": (None, [_i64, _i64, _f64, _f64, _pf, _pf, _i64]),
        "orc_hier_1d_f32": (None, [_i64, _f64, _pf, _pf, _i64, _i64, _i64, _i64]),
        "orc_hier_2d_f32": (None, [_i64, _i64, _f64, _f64, _pf, _pf, _i64, _i64, _i64, _i64, _i64, _i64]),
        "orc_residual_1d": (_f64, [_i64, _f64, _pd, _pd, _pd]),
        "orc_residual_2d": (_f64, [_i64, _i64, _f64, _f64, _pd, _pd, _pd]),
        "orc_solve_1d": (_i64, [_i64, _f64, _pd, _pd, _i32, _i64, _i64, _i64, _f64, _i64, _pd, _pd]),
        "orc_solve_2d": (_i64, [_i64, _i64, _f64, _f64, _pd, _pd, _i32, _i64, _i64, _i64, _i64,
                                _i64, _f64, _i64, _pd, _pd]),
        "orc_num_threads": (_i32, []),
        "orc_vc_apply_2d": (None, [_i64, _i64, _f64, _f64, _pd, _pd, _pd]),
        "orc_vc_residual_2d": (_f64, [_i64, _i64, _f64, _f64, _pd, _pd, _pd, _pd]),
        "orc_vc_solve_2d": (_i64, [_i64, _i64, _f64, _f64, _pd, _pd, _pd, _i32, _i64, _i64, _i64,
                                   _i64, _i64, _f64, _i64, _pd, _pd]),
        "orc_vc_grad_a_2d": (None, [_i64, _i64, _f64, _f64, _pd, _pd, _pd]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _arr(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p(a):
    return a.ctypes.data_as(_pd)


def _arr32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _p32(a):
    return a.ctypes.data_as(_pf)


def num_threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().orc_num_threads())


# ---------------------------------------------------------------- partition

def axis_tiles(n, t, o=0):
    """Tiles along one axis: list of (start, owned_lo, owned_hi)."""
    lib = _load()
    nt = lib.orc_axis_ntiles(n, t, o)
    out = []
    for i in range(nt):
        lo, hi = _i64(), _i64()
        lib.orc_axis_owned(n, t, o, i, ctypes.byref(lo), ctypes.byref(hi))
        out.append((int(lib.orc_axis_start(n, t, o, i)), lo.value, hi.value))
    return out


# ---------------------------------------------------------------- 1D

def jacobi_1d(f, x0, h, nsweeps):
    f = _arr(f)
    x = _arr(x0, f.shape).copy()
    _load().orc_jacobi_1d(f.size, h, _p(f), _p(x), int(nsweeps))
    return x


def hier_1d(f, x0, h, tile, s, ncycles, overlap=0):
    f = _arr(f)
    x = _arr(x0, f.shape).copy()
    _check_tile(tile, overlap, s)
    _load().orc_hier_1d(f.size, h, _p(f), _p(x), int(tile), int(overlap), int(s), int(ncycles))
    return x


def residual_1d(f, x, h):
    f = _arr(f)
    x = _arr(x, f.shape)
    r = np.empty_like(f)
    nrm = _load().orc_residual_1d(f.size, h, _p(f), _p(x), _p(r))
    return r, float(nrm)


def solve_1d(f, x0, h, method=HIERARCHICAL, tile=32, s=16, tol=1e-6, max_cycles=10**6, overlap=0):
    """Returns (x, cycles or -1, rel_residual, r0_norm)."""
    f = _arr(f)
    x = _arr(x0, f.shape).copy()
    if method == HIERARCHICAL:
        _check_tile(tile, overlap, s)
    rel, r0 = _f64(), _f64()
    c = _load().orc_solve_1d(f.size, h, _p(f), _p(x), int(method), int(tile), int(overlap), int(s),
                             float(tol), int(max_cycles), ctypes.byref(rel), ctypes.byref(r0))
    return x, int(c), rel.value, r0.value


# ---------------------------------------------------------------- 2D

def jacobi_2d(f, x0, hx, hy, nsweeps):
    f = _arr(f)
    ny, nx = f.shape
    x = _arr(x0, f.shape).copy()
    _load().orc_jacobi_2d(nx, ny, hx, hy, _p(f), _p(x), int(nsweeps))
    return x


def hier_2d(f, x0, hx, hy, tile, s, ncycles, overlap=(0, 0)):
    """tile = (tile_x, tile_y); overlap = (o_x, o_y)."""
    f = _arr(f)
    ny, nx = f.shape
    x = _arr(x0, f.shape).copy()
    tx, ty = tile
    ox, oy = overlap
    _check_tile(tx, ox, s)
    _check_tile(ty, oy, s)
    _load().orc_hier_2d(nx, ny, hx, hy, _p(f), _p(x), tx, ty, ox, oy, int(s), int(ncycles))
    return x


# ---------------------------------------------------------------- FP32
# The same sweeps and cycles in single precision (readings in the C source):
# inputs are rounded to float32 first; results are float32 arrays.

def jacobi_1d_f32(f, x0, h, nsweeps):
    f = _arr32(f)
    x = _arr32(x0, f.shape).copy()
    _load().orc_jacobi_1d_f32(f.size, h, _p32(f), _p32(x), int(nsweeps))
    return x


def hier_1d_f32(f, x0, h, tile, s, ncycles, overlap=0):
    f = _arr32(f)
    x = _arr32(x0, f.shape).copy()
    _check_tile(tile, overlap, s)
    _load().orc_hier_1d_f32(f.size, h, _p32(f), _p32(x), int(tile), int(overlap), int(s), int(ncycles))
    return x


def jacobi_2d_f32(f, x0, hx, hy, nsweeps):
    f = _arr32(f)
    ny, nx = f.shape
    x = _arr32(x0, f.shape).copy()
    _load().orc_jacobi_2d_f32(nx, ny, hx, hy, _p32(f), _p32(x), int(nsweeps))
    return x


def hier_2d_f32(f, x0, hx, hy, tile, s, ncycles, overlap=(0, 0)):
    f = _arr32(f)
    ny, nx = f.shape
    x = _arr32(x0, f.shape).copy()
    tx, ty = tile
    ox, oy = overlap
    _check_tile(tx, ox, s)
    _check_tile(ty, oy, s)
    _load().orc_hier_2d_f32(nx, ny, hx, hy, _p32(f), _p32(x), tx, ty, ox, oy, int(s), int(ncycles))
    return x


def residual_2d(f, x, hx, hy):
    f = _arr(f)
    ny, nx = f.shape
    x = _arr(x, f.shape)
    r = np.empty_like(f)
    nrm = _load().orc_residual_2d(nx, ny, hx, hy, _p(f), _p(x), _p(r))
    return r, float(nrm)


def solve_2d(f, x0, hx, hy, method=HIERARCHICAL, tile=(32, 32), s=16, tol=1e-6,
             max_cycles=10**6, overlap=(0, 0)):
    """Returns (x, cycles or -1, rel_residual, r0_norm)."""
    f = _arr(f)
    ny, nx = f.shape
    x = _arr(x0, f.shape).copy()
    tx, ty = tile
    ox, oy = overlap
    if method == HIERARCHICAL:
        _check_tile(tx, ox, s)
        _check_tile(ty, oy, s)
    rel, r0 = _f64(), _f64()
    c = _load().orc_solve_2d(nx, ny, hx, hy, _p(f), _p(x), int(method), tx, ty, ox, oy, int(s),
                             float(tol), int(max_cycles), ctypes.byref(rel), ctypes.byref(r0))
    return x, int(c), rel.value, r0.value


# ---------------------------------------------------------------- variable coefficients
# a: node coefficients on the (ny+2, nx+2) grid including boundary nodes.

def _a_arr(a, ny, nx):
    return _arr(a, (ny + 2, nx + 2))


def vc_apply_2d(a, u, hx, hy):
    """A(a) u for -div(a grad u) with arithmetic-mean face coefficients."""
    u = _arr(u)
    ny, nx = u.shape
    a = _a_arr(a, ny, nx)
    out = np.empty_like(u)
    _load().orc_vc_apply_2d(nx, ny, hx, hy, _p(a), _p(u), _p(out))
    return out


def vc_residual_2d(a, f, u, hx, hy):
    f = _arr(f)
    ny, nx = f.shape
    a = _a_arr(a, ny, nx)
    u = _arr(u, f.shape)
    r = np.empty_like(f)
    nrm = _load().orc_vc_residual_2d(nx, ny, hx, hy, _p(a), _p(f), _p(u), _p(r))
    return r, float(nrm)


def vc_solve_2d(a, f, x0, hx, hy, method=HIERARCHICAL, tile=(32, 32), s=8, tol=1e-10,
                max_cycles=10**6, overlap=(0, 0)):
    """Returns (x, cycles or -1, rel_residual, r0_norm); tol <= 0 runs max_cycles cycles."""
    f = _arr(f)
    ny, nx = f.shape
    a = _a_arr(a, ny, nx)
    x = _arr(x0, f.shape).copy()
    tx, ty = tile
    ox, oy = overlap
    if method == HIERARCHICAL:
        _check_tile(tx, ox, s)
        _check_tile(ty, oy, s)
    rel, r0 = _f64(), _f64()
    c = _load().orc_vc_solve_2d(nx, ny, hx, hy, _p(a), _p(f), _p(x), int(method), tx, ty, ox, oy,
                                int(s), float(tol), int(max_cycles), ctypes.byref(rel),
                                ctypes.byref(r0))
    return x, int(c), rel.value, r0.value


def vc_grad_a_2d(u, lam, hx, hy):
    """dL/da for A(a) u = f given the adjoint lam (A lam = dL/du)."""
    u = _arr(u)
    ny, nx = u.shape
    lam = _arr(lam, u.shape)
    g = np.empty((ny + 2, nx + 2))
    _load().orc_vc_grad_a_2d(nx, ny, hx, hy, _p(u), _p(lam), _p(g))
    return g


def _check_tile(t, o, s):
    if t < 1 or o < 0 or o >= t or s < 1:
        raise ValueError(f"invalid tile={t} overlap={o} s={s}")
