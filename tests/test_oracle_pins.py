"""Pins for the CPU FP64 oracle: facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself:
closed-form eigen-decay of the Jacobi iteration (Sec. 2.1 convergence
condition, Poisson spectra), exact classical iterates in the eigenbasis,
the paper's statement that one sub-iteration per cycle is plain Jacobi
(Sec. 3.3), a single tile being plain Jacobi, a dense brute-force build of the
cycle operator from the three steps of Sec. 3.3 / 4.1 with the overlap rule of
Sec. 3.5 / 4.3, the direct banded solve the paper names (Thomas, Sec. 3), a
sparse-matrix residual, affinity, and a hand-worked example.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from paper_2006_16465_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
# Independent constructions used only by these pins.

def sine_vec_1d(n, k):
    x = np.arange(1, n + 1) / (n + 1)
    return np.sin(np.pi * k * x)


def sine_vec_2d(nx, ny, k, l):
    return np.outer(sine_vec_1d(ny, l), sine_vec_1d(nx, k))


def poisson_matrix_1d(n, h):
    main = np.full(n, 2.0)
    off = np.full(n - 1, -1.0)
    return sp.diags([off, main, off], [-1, 0, 1]) / (h * h)


def poisson_matrix_2d(nx, ny, hx, hy):
    ax = poisson_matrix_1d(nx, hx)
    ay = poisson_matrix_1d(ny, hy)
    # row-major [ny, nx]: x varies fastest
    return (sp.kron(sp.identity(ny), ax) + sp.kron(ay, sp.identity(nx))).tocsr()


def tiles_by_distance(n, t, o):
    """Partition of one axis written from the paper's ownership statement:
    full tiles of t points at stride t - o (the last one moved to end at n),
    and each point written by the covering tile where it is farthest from a
    frozen subdomain edge (domain walls are not frozen); ties go left."""
    if n <= t:
        return [(0, 0, n)]
    stride = t - o
    starts = []
    i = 0
    while i * stride < n - o:
        starts.append(min(i * stride, n - t))
        i += 1
    owner = []
    for p in range(n):
        best, bestd = None, None
        for ti, a in enumerate(starts):
            if not (a <= p < a + t):
                continue
            dl = p - a + 1 if a > 0 else np.inf
            dr = a + t - p if a + t < n else np.inf
            d = min(dl, dr)
            if bestd is None or d > bestd:
                best, bestd = ti, d
        owner.append(best)
    out = []
    for ti, a in enumerate(starts):
        pts = [p for p in range(n) if owner[p] == ti]
        assert pts == list(range(pts[0], pts[-1] + 1))
        out.append((a, pts[0], pts[-1] + 1))
    return out


def dense_cycle_1d(n, h, t, o, s):
    """Cycle as an affine map x' = G x + K f, assembled tile by tile:
    extract tile + one-point halo, apply s local Jacobi sweeps with the halo
    rows held fixed, keep the owned points."""
    G = np.zeros((n, n))
    K = np.zeros((n, n))
    for a, lo, hi in tiles_by_distance(n, t, o):
        ext = min(t, n)
        m = ext + 2
        E = np.zeros((m, n))          # global -> local (halo outside domain = 0)
        for j in range(-1, ext + 1):
            g = a + j
            if 0 <= g < n:
                E[j + 1, g] = 1.0
        J = np.eye(m)                 # one local sweep on the interior rows
        B = np.zeros((m, n))
        for j in range(ext):
            J[j + 1, :] = 0.0
            J[j + 1, j] = 0.5
            J[j + 1, j + 2] = 0.5
            B[j + 1, a + j] = 0.5 * h * h
        Js = np.linalg.matrix_power(J, s)
        Ks = sum(np.linalg.matrix_power(J, k) @ B for k in range(s))
        for g in range(lo, hi):
            G[g] += (Js @ E)[g - a + 1]
            K[g] += Ks[g - a + 1]
    return G, K


def dense_cycle_2d(nx, ny, hx, hy, tx, ty, ox, oy, s):
    n = nx * ny
    wx, wy = 1 / (hx * hx), 1 / (hy * hy)
    D = 2 * wx + 2 * wy
    G = np.zeros((n, n))
    K = np.zeros((n, n))
    for ar, rlo, rhi in tiles_by_distance(ny, ty, oy):
        for ac, clo, chi in tiles_by_distance(nx, tx, ox):
            ex, ey = min(tx, nx), min(ty, ny)
            px = ex + 2
            m = px * (ey + 2)
            E = np.zeros((m, n))
            for r in range(-1, ey + 1):
                for q in range(-1, ex + 1):
                    gr, gq = ar + r, ac + q
                    if 0 <= gr < ny and 0 <= gq < nx:
                        E[(r + 1) * px + q + 1, gr * nx + gq] = 1.0
            J = np.eye(m)
            B = np.zeros((m, n))
            for r in range(ey):
                for q in range(ex):
                    i = (r + 1) * px + q + 1
                    J[i, :] = 0.0
                    J[i, i - 1] = J[i, i + 1] = wx / D
                    J[i, i - px] = J[i, i + px] = wy / D
                    B[i, (ar + r) * nx + ac + q] = 1.0 / D
            Js = np.linalg.matrix_power(J, s)
            Ks = sum(np.linalg.matrix_power(J, k) @ B for k in range(s))
            JE = Js @ E
            for gr in range(rlo, rhi):
                for gq in range(clo, chi):
                    i = (gr - ar + 1) * px + gq - ac + 1
                    G[gr * nx + gq] += JE[i]
                    K[gr * nx + gq] += Ks[i]
    return G, K


def rel_err(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# ----------------------------------------------------------------- partition

@pytest.mark.parametrize("n,t,o", [(n, t, o) for n in (1, 3, 12, 13, 31, 64, 65, 100, 257)
                                   for t in (4, 8, 32) for o in range(0, t, 2) if o < t])
def test_partition_matches_farthest_from_edge_rule(orc, n, t, o):
    assert orc.axis_tiles(n, t, o) == tiles_by_distance(n, t, o)


def test_partition_counts_printed_in_paper(orc):
    g = json.load(open(os.path.join(GOLDEN, "partition_examples.json")))
    for c in g["cases_1d"]:
        assert len(orc.axis_tiles(c["n"], c["tile"], c["overlap"])) == c["blocks"], c["source"]
    for c in g["cases_2d"]:
        nb = len(orc.axis_tiles(c["nx"], c["tile"][0], c["overlap"][0])) * \
            len(orc.axis_tiles(c["ny"], c["tile"][1], c["overlap"][1]))
        assert nb == c["blocks"], c["source"]


# ----------------------------------------------------------------- P1 eigen-decay

@pytest.mark.parametrize("n,k", [(64, 1), (64, 17), (64, 64), (100, 33)])
@pytest.mark.parametrize("nsweeps", [1, 10, 1000])
def test_classical_1d_sine_mode_decays_by_cos(orc, n, k, nsweeps):
    h = 1.0 / (n + 1)
    v = sine_vec_1d(n, k)
    x = orc.jacobi_1d(np.zeros(n), v, h, nsweeps)
    mu = np.cos(np.pi * k * h)
    assert np.max(np.abs(x - mu ** nsweeps * v)) <= 1e-13 * max(1.0, nsweeps ** 0.5)


@pytest.mark.parametrize("nx,ny,k,l", [(32, 32, 1, 1), (32, 32, 5, 30), (40, 24, 7, 3)])
@pytest.mark.parametrize("nsweeps", [1, 10, 1000])
def test_classical_2d_sine_mode_decay(orc, nx, ny, k, l, nsweeps):
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    v = sine_vec_2d(nx, ny, k, l)
    x = orc.jacobi_2d(np.zeros((ny, nx)), v, hx, hy, nsweeps)
    wx, wy = 1 / hx ** 2, 1 / hy ** 2
    mu = (wx * np.cos(np.pi * k * hx) + wy * np.cos(np.pi * l * hy)) / (wx + wy)
    assert np.max(np.abs(x - mu ** nsweeps * v)) <= 1e-13 * max(1.0, nsweeps ** 0.5)


# ----------------------------------------------------------------- P2 closed-form iterates

def spectral_1d(n, seed, n_modes=8):
    rng = np.random.default_rng(seed)
    k = rng.integers(1, n + 1, n_modes)
    a = rng.standard_normal(n_modes)
    h = 1.0 / (n + 1)
    lam = 4 / h ** 2 * np.sin(np.pi * k * h / 2) ** 2
    mu = 1 - lam / (2 / h ** 2)
    return k, a, lam, mu, h


def closed_form_count(amps, mus, tol):
    """smallest n with ||sum_g A_g mu_g^n v_g|| <= tol ||sum_g A_g v_g|| for
    orthogonal v_g of equal norm (discrete sine modes)."""
    A2 = np.asarray(amps) ** 2
    mus = np.asarray(mus)
    target = tol * tol * A2.sum()
    n = 0
    while (A2 * mus ** (2 * n)).sum() > target:
        n += 1
    return n


def group_modes(keys, a, mu):
    d = {}
    for key, am, m in zip(keys, a, mu):
        A, _ = d.get(key, (0.0, m))
        d[key] = (A + am, m)
    return [v[0] for v in d.values()], [v[1] for v in d.values()]


def test_classical_1d_iterates_match_eigen_expansion(orc):
    n = 256
    k, a, lam, mu, h = spectral_1d(n, 3)
    f = W.rhs_1d_modes(n, 8, 3)
    for ns in (1, 7, 50, 400):
        x = orc.jacobi_1d(f, np.zeros(n), h, ns)
        xe = sum(am * (1 - mm ** ns) / lm * sine_vec_1d(n, km) for km, am, lm, mm in zip(k, a, lam, mu))
        assert rel_err(x, xe) <= 1e-12
        r, nrm = orc.residual_1d(f, x, h)
        re = sum(am * mm ** ns * sine_vec_1d(n, km) for km, am, mm in zip(k, a, mu))
        assert np.max(np.abs(r - re)) <= 1e-9 * np.max(np.abs(f))


@pytest.mark.parametrize("seed", range(5))
def test_classical_1d_sweeps_to_tol_match_closed_form(orc, seed):
    n = 256
    k, a, lam, mu, h = spectral_1d(n, seed)
    amps, mus = group_modes(list(k), a, mu)
    want = closed_form_count(amps, mus, 1e-6)
    f = W.rhs_1d_modes(n, 8, seed)
    _, got, rel, _ = orc.solve_1d(f, np.zeros(n), h, method=orc.CLASSICAL, tol=1e-6)
    assert got == want
    assert rel <= 1e-6


@pytest.mark.parametrize("n,seed", [(256, 0), (256, 1), (4096, 0)])
def test_classical_2d_sweeps_to_tol_match_closed_form(orc, n, seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(1, n + 1, 8)
    l = rng.integers(1, n + 1, 8)
    a = rng.standard_normal(8)
    h = 1.0 / (n + 1)
    mu = (np.cos(np.pi * k * h) + np.cos(np.pi * l * h)) / 2
    amps, mus = group_modes(list(zip(k, l)), a, mu)
    want = closed_form_count(amps, mus, 1e-6)
    f = W.rhs_2d_modes(n, n, 8, 0.0, seed)
    _, got, rel, _ = orc.solve_2d(f, np.zeros_like(f), h, h, method=orc.CLASSICAL, tol=1e-6,
                                  max_cycles=100000)
    assert got == want
    assert rel <= 1e-6


# ----------------------------------------------------------------- P3 / P4: reductions to plain Jacobi

@pytest.mark.parametrize("n,t,o", [(256, 32, 0), (100, 32, 0), (100, 32, 4), (37, 8, 2)])
def test_one_subiteration_is_plain_jacobi_1d(orc, n, t, o):
    f = W.rhs_random(n, 1)
    x0 = W.rhs_random(n, 2)
    h = 1.0 / (n + 1)
    for nc in (1, 5, 33):
        assert np.array_equal(orc.hier_1d(f, x0, h, t, 1, nc, o), orc.jacobi_1d(f, x0, h, nc))


@pytest.mark.parametrize("nx,ny,tile,ov,hx,hy", [
    (64, 64, (32, 32), (0, 0), None, None),
    (70, 45, (32, 16), (0, 0), None, None),
    (70, 45, (16, 8), (4, 2), None, None),
    (50, 40, (16, 16), (0, 0), 0.02, 0.03),
])
def test_one_subiteration_is_plain_jacobi_2d(orc, nx, ny, tile, ov, hx, hy):
    hx = hx or 1.0 / (nx + 1)
    hy = hy or 1.0 / (ny + 1)
    f = W.rhs_random((ny, nx), 3)
    x0 = W.rhs_random((ny, nx), 4)
    for nc in (1, 6):
        assert np.array_equal(orc.hier_2d(f, x0, hx, hy, tile, 1, nc, ov), orc.jacobi_2d(f, x0, hx, hy, nc))


def test_single_tile_is_s_plain_sweeps(orc):
    n = 40
    h = 1.0 / (n + 1)
    f = W.rhs_random(n, 5)
    x0 = W.rhs_random(n, 6)
    for s in (1, 2, 7, 16):
        assert np.array_equal(orc.hier_1d(f, x0, h, 64, s, 3), orc.jacobi_1d(f, x0, h, 3 * s))
    f2 = W.rhs_random((20, 30), 7)
    x2 = W.rhs_random((20, 30), 8)
    for s in (1, 3, 8):
        assert np.array_equal(orc.hier_2d(f2, x2, 0.03, 0.03, (32, 32), s, 2),
                              orc.jacobi_2d(f2, x2, 0.03, 0.03, 2 * s))


@pytest.mark.parametrize("shape", [(77, 100), (64, 130), (200, 33)])
@pytest.mark.parametrize("tile", [(32, 32), (64, 32), (16, 16)])
def test_overlap_beyond_halo_reach_is_exactly_classical(orc, shape, tile):
    """A frozen edge value is stale from the second sub-iteration on, and the
    error it injects moves one point per sweep, so after s sweeps the points at
    distance >= s from every frozen edge carry exact classical iterates.  The
    overlap rule (Sec. 3.5 / 4.3) puts the owned points ceil(o/2) + 1 away from
    the edges: with o >= 2s - 2 a cycle is exactly s classical sweeps, and with
    o = 2s - 3 it is not.  Pins the halo freezing and the ownership split."""
    ny, nx = shape
    f = W.rhs_random(shape, 3)
    x0 = W.rhs_random(shape, 4)
    h = 1.0 / (max(shape) + 1)
    for s in (1, 2, 3, 4, 5, 8):
        o = 2 * s - 2
        if o >= min(tile):
            continue
        want = orc.jacobi_2d(f, x0, h, h, 3 * s)
        for oo in (o, o + 1):
            if oo < min(tile):
                assert np.array_equal(orc.hier_2d(f, x0, h, h, tile, s, 3, (oo, oo)), want)
        if s >= 2:
            assert not np.array_equal(orc.hier_2d(f, x0, h, h, tile, s, 3, (o - 1, o - 1)), want)


def test_overlap_beyond_halo_reach_1d(orc):
    n = 333
    f, x0 = W.rhs_random(n, 5), W.rhs_random(n, 6)
    h = 1.0 / (n + 1)
    for t in (32, 64):
        for s in (2, 4, 7):
            want = orc.jacobi_1d(f, x0, h, 4 * s)
            assert np.array_equal(orc.hier_1d(f, x0, h, t, s, 4, 2 * s - 2), want)
            assert not np.array_equal(orc.hier_1d(f, x0, h, t, s, 4, 2 * s - 3), want)


# ----------------------------------------------------------------- P6: dense brute force

# Sec. 3.5, Table 2: for each k, the overlap that gave the least time on the
# paper's 1D experiment (1024 interior points, b = 1, x0 = 1, residual reduced
# by 1e-4, 32-point subdomains, even overlaps up to 30).
TABLE2_OPTIMAL_OVERLAP = {4: 2, 8: 4, 16: 4, 32: 8, 64: 10, 128: 12}


@pytest.mark.parametrize("k", sorted(TABLE2_OPTIMAL_OVERLAP))
def test_overlap_cost_model_reproduces_table2(orc, k):
    """Time per cycle grows with the operational-block count of Sec. 3.5,
    (N - o) / (tpb - o) (the blocks the partition rule yields), at a fixed
    cost per block for a given k; the time to tolerance is therefore
    proportional to cycles(o) x blocks(o).  Its minimum over the even
    overlaps 0..30 on the paper's own 1D experiment must fall on the optimal
    overlap of Table 2 for every k: pins the overlap partition and the
    ownership split against the paper's measured optimum (the cycle counts
    come from the oracle, nothing is fitted)."""
    n = 1024
    h = 1.0 / (n + 1)
    f, x0 = np.ones(n), np.ones(n)
    cost = {}
    for o in range(0, 31, 2):
        _, cycles, rel_, _ = orc.solve_1d(f, x0, h, tile=32, s=k, tol=1e-4, overlap=o)
        assert rel_ <= 1e-4
        blocks = len(orc.axis_tiles(n, 32, o))
        assert blocks == -(-(n - o) // (32 - o))  # ceil((N - o) / (tpb - o))
        cost[o] = cycles * blocks
    assert min(cost, key=cost.get) == TABLE2_OPTIMAL_OVERLAP[k], cost


@pytest.mark.parametrize("n,t,o,s", [(8, 4, 0, 1), (8, 4, 0, 2), (8, 4, 0, 3), (8, 4, 0, 5),
                                     (11, 4, 0, 3), (11, 4, 2, 3), (13, 6, 2, 4), (20, 8, 4, 6),
                                     (9, 16, 0, 3)])
def test_hier_1d_matches_dense_cycle_operator(orc, n, t, o, s):
    h = 1.0 / (n + 1)
    G, K = dense_cycle_1d(n, h, t, o, s)
    f = W.rhs_random(n, 11)
    x = W.rhs_random(n, 12)
    xd = x.copy()
    for nc in range(1, 21):
        xd = G @ xd + K @ f
        if nc in (1, 2, 5, 20):
            assert rel_err(orc.hier_1d(f, x, h, t, s, nc, o), xd) <= 1e-14
    # iteration converges (rho(G) < 1) and its fixed point solves A x = f
    assert np.max(np.abs(np.linalg.eigvals(G))) < 1.0
    xs = np.linalg.solve(np.eye(n) - G, K @ f)
    assert rel_err(xs, np.linalg.solve(poisson_matrix_1d(n, h).toarray(), f)) <= 1e-10


@pytest.mark.parametrize("nx,ny,tile,ov,s,hx,hy", [
    (6, 6, (3, 3), (0, 0), 2, None, None),
    (6, 6, (3, 3), (0, 0), 1, None, None),
    (7, 5, (3, 2), (0, 0), 3, None, None),
    (9, 7, (4, 4), (2, 2), 3, None, None),
    (6, 5, (4, 3), (0, 0), 2, 0.1, 0.2),
])
def test_hier_2d_matches_dense_cycle_operator(orc, nx, ny, tile, ov, s, hx, hy):
    hx = hx or 1.0 / (nx + 1)
    hy = hy or 1.0 / (ny + 1)
    G, K = dense_cycle_2d(nx, ny, hx, hy, tile[0], tile[1], ov[0], ov[1], s)
    f = W.rhs_random((ny, nx), 13)
    x = W.rhs_random((ny, nx), 14)
    xd = x.ravel().copy()
    for nc in range(1, 13):
        xd = G @ xd + K @ f.ravel()
        if nc in (1, 2, 12):
            got = orc.hier_2d(f, x, hx, hy, tile, s, nc, ov).ravel()
            assert rel_err(got, xd) <= 1e-14
    assert np.max(np.abs(np.linalg.eigvals(G))) < 1.0
    xs = np.linalg.solve(np.eye(nx * ny) - G, K @ f.ravel())
    A = poisson_matrix_2d(nx, ny, hx, hy).toarray()
    assert rel_err(xs, np.linalg.solve(A, f.ravel())) <= 1e-10


# ----------------------------------------------------------------- P5: converged state vs direct solves

def test_converged_1d_matches_thomas(orc):
    n = 64
    h = 1.0 / (n + 1)
    f = W.rhs_1d_modes(n, 8, 2)
    ab = np.zeros((3, n))
    ab[0, 1:] = -1 / h ** 2
    ab[1, :] = 2 / h ** 2
    ab[2, :-1] = -1 / h ** 2
    xstar = scipy.linalg.solve_banded((1, 1), ab, f)
    tol = 1e-11
    x, c, rel, r0 = orc.solve_1d(f, np.zeros(n), h, tile=16, s=8, tol=tol, max_cycles=10 ** 6)
    assert c > 0 and rel <= tol
    lam_min = 4 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    assert np.linalg.norm(x - xstar) <= tol * np.linalg.norm(f) / lam_min * 1.01 + 1e-14


def test_converged_2d_matches_direct_solve(orc):
    n = 24
    h = 1.0 / (n + 1)
    f = W.rhs_2d_modes(n, n, 8, 0.1, 1)
    A = poisson_matrix_2d(n, n, h, h)
    xstar = scipy.sparse.linalg.spsolve(A.tocsc(), f.ravel())
    tol = 1e-10
    x, c, rel, _ = orc.solve_2d(f, np.zeros_like(f), h, h, tile=(8, 8), s=4, tol=tol, overlap=(2, 2))
    assert c > 0 and rel <= tol
    lam_min = 8 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    assert np.linalg.norm(x.ravel() - xstar) <= tol * np.linalg.norm(f) / lam_min * 1.01 + 1e-14


# ----------------------------------------------------------------- residual vs sparse operator

def test_residual_matches_sparse_operator(orc):
    n = 300
    h = 1.0 / (n + 1)
    f, x = W.rhs_random(n, 21), W.rhs_random(n, 22)
    r, nrm = orc.residual_1d(f, x, h)
    rr = f - poisson_matrix_1d(n, h) @ x
    assert rel_err(r, rr) <= 1e-13
    assert abs(nrm - np.linalg.norm(rr)) <= 1e-13 * np.linalg.norm(rr)
    nx, ny, hx, hy = 37, 29, 0.02, 0.035
    f2, x2 = W.rhs_random((ny, nx), 23), W.rhs_random((ny, nx), 24)
    r2, n2 = orc.residual_2d(f2, x2, hx, hy)
    rr2 = f2.ravel() - poisson_matrix_2d(nx, ny, hx, hy) @ x2.ravel()
    assert rel_err(r2.ravel(), rr2) <= 1e-13
    assert abs(n2 - np.linalg.norm(rr2)) <= 1e-13 * np.linalg.norm(rr2)


# ----------------------------------------------------------------- P8 affinity

def test_cycle_is_affine(orc):
    nx, ny = 45, 38
    h = 1.0 / 46
    rs = [W.rhs_random((ny, nx), s) for s in (31, 32, 33, 34)]
    f, g, x, y = rs
    al, be = 0.75, -1.5
    lhs = orc.hier_2d(al * f + be * g, al * x + be * y, h, h, (16, 8), 5, 3, (2, 2))
    rhs = al * orc.hier_2d(f, x, h, h, (16, 8), 5, 3, (2, 2)) + be * orc.hier_2d(g, y, h, h, (16, 8), 5, 3, (2, 2))
    assert rel_err(lhs, rhs) <= 1e-14


# ----------------------------------------------------------------- worked example (hand-derived)

def test_worked_example_exact(orc):
    g = json.load(open(os.path.join(GOLDEN, "worked_example_1d.json")))
    n, h = 8, 1.0 / 9
    f = np.ones(n)

    def y(key):
        return np.array([float(Fraction(p, q)) for p, q in g["expected_y"][key]])

    scale = 1.0 / (h * h)
    cases = {
        "s3_cycle1": orc.hier_1d(f, np.zeros(n), h, 4, 3, 1),
        "s3_cycle2": orc.hier_1d(f, np.zeros(n), h, 4, 3, 2),
        "s1_cycle1": orc.hier_1d(f, np.zeros(n), h, 4, 1, 1),
        "s1_cycle2": orc.hier_1d(f, np.zeros(n), h, 4, 1, 2),
        "classical3": orc.jacobi_1d(f, np.zeros(n), h, 3),
    }
    for key, got in cases.items():
        assert np.max(np.abs(got * scale - y(key))) <= 1e-14 * 4, key
    # one tile of 8 points with k = 3 is exactly three classical sweeps
    assert np.array_equal(orc.hier_1d(f, np.zeros(n), h, 8, 3, 1), cases["classical3"])


def test_solve_reports_initial_residual_and_zero_rhs(orc):
    n = 50
    h = 1.0 / 51
    x, c, rel, r0 = orc.solve_1d(np.zeros(n), np.zeros(n), h, tol=1e-6)
    assert c == 0 and rel == 0.0 and r0 == 0.0
    f = W.rhs_1d_modes(n, 8, 0)
    x, c, rel, r0 = orc.solve_1d(f, np.zeros(n), h, tol=1e-6, max_cycles=3)
    assert c == -1 and rel > 1e-6
    assert abs(r0 - np.linalg.norm(f)) <= 1e-14 * np.linalg.norm(f)
