"""Seeded synthetic Poisson workloads (inputs only, no solver arithmetic).

This module is the one piece shared by the GPU path's tests/benchmark and the
CPU oracle: it draws right-hand sides and starting vectors and nothing else.

The paper's own runs use b = 1 and x0 = 1 (Sec. 3.4 for 1D with N = 1024;
Sec. 4.2 for 2D with 1024 x 1024), i.e. a smooth right-hand side.  The
workloads below add seeded random-mode right-hand sides:

* 1D: f_i = sum_m a_m sin(pi k_m x_i), x_i = i h, h = 1/(n+1), with
  k_m drawn uniformly from {1..n} (repeats allowed) and a_m ~ N(0, 1).
* 2D: f_ij = sum_m a_m sin(pi l_m y_i) sin(pi k_m x_j) (+ optional white
  noise), k_m uniform in {1..nx}, l_m uniform in {1..ny}, a_m ~ N(0, 1).

Draw order from ``numpy.random.default_rng(seed)`` (PCG64): 1D k then a;
2D k, then l, then a, then the noise field (ny, nx).  Arrays are float64 and
row-major ``[ny, nx]`` in 2D (row = y index).
"""
from __future__ import annotations

import numpy as np


def grid_h(n: int) -> float:
    """Uniform spacing on [0, 1] with n interior points: h = 1/(n+1)."""
    return 1.0 / (n + 1)


def rhs_1d_modes(n: int, n_modes: int = 8, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    k = rng.integers(1, n + 1, n_modes)
    a = rng.standard_normal(n_modes)
    x = np.arange(1, n + 1, dtype=np.float64) * grid_h(n)
    f = np.zeros(n, dtype=np.float64)
    for km, am in zip(k, a):
        f += am * np.sin(np.pi * km * x)
    return f


def rhs_2d_modes(nx: int, ny: int | None = None, n_modes: int = 8, noise_std: float = 0.0,
                 seed: int = 0) -> np.ndarray:
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    k = rng.integers(1, nx + 1, n_modes)
    l = rng.integers(1, ny + 1, n_modes)
    a = rng.standard_normal(n_modes)
    xs = np.arange(1, nx + 1, dtype=np.float64) * grid_h(nx)
    ys = np.arange(1, ny + 1, dtype=np.float64) * grid_h(ny)
    f = np.zeros((ny, nx), dtype=np.float64)
    for km, lm, am in zip(k, l, a):
        f += am * np.outer(np.sin(np.pi * lm * ys), np.sin(np.pi * km * xs))
    if noise_std > 0.0:
        f += rng.normal(0.0, noise_std, (ny, nx))
    return f


def grf_2d(n_nodes_y: int, n_nodes_x: int, length: float = 0.05, variance: float = 1.0,
           h: float | None = None, seed: int = 0) -> np.ndarray:
    """Gaussian random field with squared-exponential covariance
    variance * exp(-r^2 / (2 length^2)) on a grid of n_nodes_y x n_nodes_x nodes
    with spacing h (default 1 / (n_nodes_x - 1)): white noise filtered by the
    square root of the spectral density (periodic FFT), scaled to the target
    variance."""
    h = 1.0 / (n_nodes_x - 1) if h is None else h
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n_nodes_y, n_nodes_x))
    ky = np.fft.fftfreq(n_nodes_y, d=h)
    kx = np.fft.fftfreq(n_nodes_x, d=h)
    filt = np.exp(-np.pi ** 2 * length ** 2 * (ky[:, None] ** 2 + kx[None, :] ** 2))
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    var_theory = np.sum(filt ** 2) / (n_nodes_x * n_nodes_y)
    return g * np.sqrt(variance / var_theory)


def diffusion_coefficient(n: int, length: float = 0.05, variance: float = 1.0, seed: int = 0):
    """a = exp(g) on the (n+2) x (n+2) node grid (boundary nodes included)."""
    return np.exp(grf_2d(n + 2, n + 2, length, variance, 1.0 / (n + 1), seed))


def smooth_modes_2d(n: int, n_modes: int = 4, kmax: int = 4, seed: int = 0) -> np.ndarray:
    """sum of n_modes products sin(pi k x) sin(pi l y), k, l uniform in 1..kmax, N(0,1) amplitudes"""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, n_modes)
    l = rng.integers(1, kmax + 1, n_modes)
    a = rng.standard_normal(n_modes)
    xs = np.arange(1, n + 1) * grid_h(n)
    u = np.zeros((n, n))
    for km, lm, am in zip(k, l, a):
        u += am * np.outer(np.sin(np.pi * lm * xs), np.sin(np.pi * km * xs))
    return u


def rhs_random(shape, seed: int = 0) -> np.ndarray:
    """Unstructured N(0,1) values, for parity cases on arbitrary shapes."""
    return np.random.default_rng(seed).standard_normal(shape)


def batch_specs(seed: int = 0, n2d: int = 512, n1d: int = 128, side=(64, 1024),
                n1=(1_000, 1_000_000)):
    """The batched workload: n2d square 2D grids with side log-uniform in
    [side[0], side[1]] and n1d 1D grids with N log-uniform in [n1[0], n1[1]]
    (sizes drawn from default_rng(seed), 2D sides first, then 1D sizes).
    Returns (dim, n, rhs_seed) per problem: problem i's right-hand side is
    rhs_2d_modes(n, n, 8, 0, rhs_seed) or rhs_1d_modes(n, 8, rhs_seed), with
    rhs_seed = 1_000_003 * seed + i, so one problem can be rebuilt alone."""
    rng = np.random.default_rng(seed)
    sides = np.exp(rng.uniform(np.log(side[0]), np.log(side[1]), n2d)).astype(np.int64)
    ns = np.exp(rng.uniform(np.log(n1[0]), np.log(n1[1]), n1d)).astype(np.int64)
    sides = np.clip(sides, side[0], side[1])
    ns = np.clip(ns, n1[0], n1[1])
    out = [(2, int(n), 1_000_003 * seed + i) for i, n in enumerate(sides)]
    out += [(1, int(n), 1_000_003 * seed + n2d + i) for i, n in enumerate(ns)]
    return out


def batch_rhs(spec) -> np.ndarray:
    dim, n, sd = spec
    return rhs_2d_modes(n, n, 8, 0.0, sd) if dim == 2 else rhs_1d_modes(n, 8, sd)


# Named workloads.  "tile" is (tile_x, tile_y) in 2D, an int in 1D.
CONFIGS = {
    # 1D Poisson, N = 256, 8 random sine modes, tile 32, s = 16, to 1e-6
    "poisson1d_n256": dict(dim=1, n=256, n_modes=8, noise_std=0.0, tile=32, s=16, tol=1e-6),
    # 2D 512 x 512, 16 separable modes + N(0, 0.01) white noise (sigma 0.1),
    # 32 x 32 tiles, s in {1, 4, 8, 16, 32}, to 1e-6
    "poisson2d_512": dict(dim=2, n=512, n_modes=16, noise_std=0.1, tile=(32, 32),
                          s_grid=(1, 4, 8, 16, 32), s=16, tol=1e-6),
    # 2D 4096 x 4096, 8 separable modes, no noise, to 1e-6 (time-to-tolerance workload)
    "poisson2d_4096": dict(dim=2, n=4096, n_modes=8, noise_std=0.0, tile=(32, 32), s=16, tol=1e-6),
}


def make(config: str, seed: int = 0):
    """Return (f, h) for a named configuration."""
    c = CONFIGS[config]
    if c["dim"] == 1:
        return rhs_1d_modes(c["n"], c["n_modes"], seed), grid_h(c["n"])
    return rhs_2d_modes(c["n"], c["n"], c["n_modes"], c["noise_std"], seed), grid_h(c["n"])
