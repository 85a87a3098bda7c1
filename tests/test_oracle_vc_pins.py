"""Pins for the variable-coefficient part of the CPU oracle: the operator
-div(a grad u) with arithmetic-mean face coefficients (the general pentadiagonal
Jacobi setting of Sec. 4 with per-point coefficients), its Jacobi and
hierarchical iterations, and the adjoint gradient with respect to a.

Independent references: a sparse assembly G^T diag(a_face) G from the discrete
gradient, dense Jacobi from that matrix, sparse direct solves, and central
finite differences of a loss evaluated with direct solves."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2006_16465_amd import workloads as W


def assemble(a, nx, ny, hx, hy):
    """A = Gx^T diag(ax) Gx / hx^2 + Gy^T diag(ay) Gy / hy^2 over all faces,
    boundary values eliminated (Dirichlet 0)."""
    p = nx + 2
    node = lambda r, q: (r + 1) * p + (q + 1)
    rows, cols, vals, face_a = [], [], [], []
    fidx = 0
    idx = lambda r, q: r * nx + q if 0 <= r < ny and 0 <= q < nx else None
    blocks = []
    for (dr, dq, h) in ((0, 1, hx), (1, 0, hy)):
        rr, cc, vv, fa = [], [], [], []
        f = 0
        for r in range(-1 if dr else 0, ny):
            for q in range(-1 if dq else 0, nx):
                if dr == 0 and not (0 <= r < ny):
                    continue
                if dq == 0 and not (0 <= q < nx):
                    continue
                i0, i1 = idx(r, q), idx(r + dr, q + dq)
                if i0 is None and i1 is None:
                    continue
                if i0 is not None:
                    rr.append(f); cc.append(i0); vv.append(1.0)
                if i1 is not None:
                    rr.append(f); cc.append(i1); vv.append(-1.0)
                fa.append(0.5 * (a.ravel()[node(r, q)] + a.ravel()[node(r + dr, q + dq)]) / (h * h))
                f += 1
        G = sp.csr_matrix((vv, (rr, cc)), shape=(f, nx * ny))
        blocks.append(G.T @ sp.diags(fa) @ G)
    return (blocks[0] + blocks[1]).tocsr()


@pytest.fixture(scope="module")
def case():
    nx, ny = 13, 9
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    a = np.exp(W.grf_2d(ny + 2, nx + 2, 0.2, 1.0, hx, seed=3))
    return nx, ny, hx, hy, a


def test_operator_matches_gradient_form_and_is_symmetric(orc, case):
    nx, ny, hx, hy, a = case
    A = assemble(a, nx, ny, hx, hy)
    u = W.rhs_random((ny, nx), 1)
    assert np.max(np.abs(orc.vc_apply_2d(a, u, hx, hy).ravel() - A @ u.ravel())) <= 1e-12 * np.max(np.abs(A @ u.ravel()))
    v, w = W.rhs_random((ny, nx), 2), W.rhs_random((ny, nx), 3)
    lhs = np.sum(v * orc.vc_apply_2d(a, w, hx, hy))
    rhs = np.sum(w * orc.vc_apply_2d(a, v, hx, hy))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_constant_coefficient_is_poisson(orc):
    nx, ny, h = 20, 20, 1.0 / 21
    a = np.full((ny + 2, nx + 2), 2.5)
    u = W.rhs_random((ny, nx), 4)
    f = W.rhs_random((ny, nx), 5)
    r_vc, _ = orc.vc_residual_2d(a, 2.5 * f, u, h, h)
    r_p, _ = orc.residual_2d(f, u, h, h)
    assert np.max(np.abs(r_vc - 2.5 * r_p)) <= 1e-12 * np.max(np.abs(r_vc))


def test_classical_sweeps_match_matrix_jacobi(orc, case):
    nx, ny, hx, hy, a = case
    A = assemble(a, nx, ny, hx, hy)
    d = A.diagonal()
    f = W.rhs_random((ny, nx), 6)
    x = W.rhs_random((ny, nx), 7).ravel()
    got = orc.vc_solve_2d(a, f, x.reshape(ny, nx), hx, hy, method=orc.CLASSICAL, tol=0.0, max_cycles=25)[0]
    for _ in range(25):
        x = x + (f.ravel() - A @ x) / d
    assert np.max(np.abs(got.ravel() - x)) <= 1e-12 * np.max(np.abs(x))


def test_one_subiteration_is_classical_and_overlap_rule_holds(orc, case):
    nx, ny, hx, hy, a = case
    f = W.rhs_random((ny, nx), 8)
    x0 = W.rhs_random((ny, nx), 9)
    cl = orc.vc_solve_2d(a, f, x0, hx, hy, method=orc.CLASSICAL, tol=0.0, max_cycles=6)[0]
    hi = orc.vc_solve_2d(a, f, x0, hx, hy, tile=(4, 4), s=1, tol=0.0, max_cycles=6)[0]
    assert np.array_equal(cl, hi)
    # overlap 2s - 2: each cycle is exactly s classical sweeps (halo never reaches owned points)
    cl9 = orc.vc_solve_2d(a, f, x0, hx, hy, method=orc.CLASSICAL, tol=0.0, max_cycles=9)[0]
    hi3 = orc.vc_solve_2d(a, f, x0, hx, hy, tile=(8, 8), s=3, overlap=(4, 4), tol=0.0, max_cycles=3)[0]
    assert np.array_equal(cl9, hi3)


def test_hierarchical_cycle_matches_dense_operator(orc, case):
    """Cycle built from the three steps with matrix rows of A as local Jacobi."""
    nx, ny, hx, hy, a = case
    A = assemble(a, nx, ny, hx, hy).toarray()
    n = nx * ny
    tx, ty, s = 5, 4, 3
    from test_oracle_pins import tiles_by_distance
    G = np.zeros((n, n))
    K = np.zeros((n, n))
    for ar, rlo, rhi in tiles_by_distance(ny, ty, 0):
        for ac, clo, chi in tiles_by_distance(nx, tx, 0):
            ex, ey = min(tx, nx), min(ty, ny)
            inside = [(r, q) for r in range(ar, ar + ey) for q in range(ac, ac + ex)]
            ii = [r * nx + q for r, q in inside]
            # local iteration on the tile's unknowns with everything else frozen at x
            M = np.eye(n)
            B = np.zeros((n, n))
            for i in ii:
                M[i, :] = -A[i, :] / A[i, i]
                M[i, i] = 0.0
                B[i, i] = 1.0 / A[i, i]
            Ms = np.linalg.matrix_power(M, s)
            Bs = sum(np.linalg.matrix_power(M, k) @ B for k in range(s))
            for r in range(rlo, rhi):
                for q in range(clo, chi):
                    G[r * nx + q] = Ms[r * nx + q]
                    K[r * nx + q] = Bs[r * nx + q]
    f = W.rhs_random((ny, nx), 10)
    x = W.rhs_random((ny, nx), 11)
    xd = x.ravel()
    for c in range(1, 6):
        xd = G @ xd + K @ f.ravel()
    got = orc.vc_solve_2d(a, f, x, hx, hy, tile=(tx, ty), s=s, tol=0.0, max_cycles=5)[0]
    assert np.max(np.abs(got.ravel() - xd)) <= 1e-12 * np.max(np.abs(xd))


def test_converged_solution_matches_direct_solve(orc, case):
    nx, ny, hx, hy, a = case
    A = assemble(a, nx, ny, hx, hy).tocsc()
    f = W.rhs_random((ny, nx), 12)
    x, c, rel, _ = orc.vc_solve_2d(a, f, np.zeros_like(f), hx, hy, tile=(8, 4), s=4, tol=1e-12)
    assert c > 0 and rel <= 1e-12
    xs = spla.spsolve(A, f.ravel())
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)


def test_adjoint_gradient_matches_finite_differences(orc):
    """L(a, f) = sum (u - t)^2 with A(a) u = f.  dL/df = lam, dL/da from the
    face-product formula; both against central differences (eps = 1e-6) of L
    evaluated with sparse direct solves."""
    nx, ny = 10, 8
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    a = np.exp(W.grf_2d(ny + 2, nx + 2, 0.2, 1.0, hx, seed=5))
    f = W.rhs_random((ny, nx), 13)
    t = W.rhs_random((ny, nx), 14) * 1e-3

    def loss(aa, ff):
        u = spla.spsolve(assemble(aa, nx, ny, hx, hy).tocsc(), ff.ravel())
        return np.sum((u - t.ravel()) ** 2)

    A = assemble(a, nx, ny, hx, hy).tocsc()
    u = spla.spsolve(A, f.ravel())
    lam = spla.spsolve(A, 2 * (u - t.ravel()))          # A symmetric: adjoint = forward solve
    ga = orc.vc_grad_a_2d(u.reshape(ny, nx), lam.reshape(ny, nx), hx, hy)
    rng = np.random.default_rng(0)
    eps = 1e-6
    for _ in range(12):
        r, q = rng.integers(0, ny + 2), rng.integers(0, nx + 2)
        ap, am = a.copy(), a.copy()
        ap[r, q] += eps
        am[r, q] -= eps
        fd = (loss(ap, f) - loss(am, f)) / (2 * eps)
        assert abs(fd - ga[r, q]) <= 1e-6 * max(1e-8, np.max(np.abs(ga))), (r, q, fd, ga[r, q])
    for _ in range(6):
        r, q = rng.integers(0, ny), rng.integers(0, nx)
        fp, fm = f.copy(), f.copy()
        fp[r, q] += eps
        fm[r, q] -= eps
        fd = (loss(a, fp) - loss(a, fm)) / (2 * eps)
        assert abs(fd - lam.reshape(ny, nx)[r, q]) <= 1e-6 * np.max(np.abs(lam))


def test_grf_statistics():
    g = W.grf_2d(258, 258, 0.05, 1.0, 1.0 / 257, seed=0)
    assert abs(np.var(g) - 1.0) <= 0.25
    # correlation at lag L: exp(-L^2 h^2 / (2 l^2)); h = 1/257, l = 0.05 -> lag 13 ~ e^-0.5
    lag = 13
    c = np.mean(g[:, :-lag] * g[:, lag:]) / np.var(g)
    assert abs(c - np.exp(-(lag / 257) ** 2 / (2 * 0.05 ** 2))) <= 0.15
