"""GPU parity for variable-coefficient diffusion -div(a grad u) = f and its
adjoint: forward iterates and cycles-to-tolerance against the CPU oracle, the
gradient with respect to a against the oracle's face-product formula (itself
pinned by finite differences of direct solves), and torch autograd through the
adjoint solve against central finite differences."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def prob():
    ny, nx = 48, 64
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    a = np.exp(W.grf_2d(ny + 2, nx + 2, 0.15, 1.0, hx, seed=7))
    f = np.stack([W.rhs_2d_modes(nx, ny, 8, 0.1, s) for s in range(3)])
    return nx, ny, hx, hy, a, f


# 64 x 48 grid: the first four shapes hold a full tile in each direction and
# run register-resident tiles by default; (16, 64) and (32, 64) are taller
# than the grid and run the LDS tile.  lds_kernel forces the LDS tile.
@pytest.mark.parametrize("lds", [False, True], ids=["default", "lds"])
@pytest.mark.parametrize("tile,s,ov", [((32, 32), 8, (0, 0)), ((16, 16), 4, (6, 6)), ((64, 16), 3, (2, 2)),
                                       ((64, 32), 8, (14, 14)), ((16, 64), 5, (8, 8)), ((32, 64), 2, (0, 0))])
def test_vc_fixed_cycles_match_oracle(orc, prob, tile, s, ov, lds):
    nx, ny, hx, hy, a, f = prob
    U = torch.zeros_like(dev(f))
    hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, tile=tile, s=s, overlap=ov, rel_tol=0.0, max_cycles=5,
                   lds_kernel=lds)
    got = host(U)
    for b in range(f.shape[0]):
        want = orc.vc_solve_2d(a, f[b], np.zeros((ny, nx)), hx, hy, tile=tile, s=s, overlap=ov,
                               tol=0.0, max_cycles=5)[0]
        assert np.array_equal(got[b], want), f"batch {b}"


@pytest.mark.parametrize("tile,s,ov", [((64, 32), 8, (14, 14)), ((32, 64), 6, (10, 10)), ((16, 32), 3, (0, 0)),
                                       ((64, 64), 4, (6, 6))])
def test_vc_register_tiles_on_a_ragged_grid_match_oracle(orc, tile, s, ov):
    """150 x 75 with anisotropic spacing: several tiles per axis with the
    last one moved left to end at the grid edge, so the ownership split
    between overlapping tiles is uneven; register-resident tiles (default)
    and the LDS tile must both give the oracle's iterates bit for bit, after
    fixed cycles and at the tolerance (the residual fused into the load)."""
    nx, ny = 150, 75
    hx, hy = 1.0 / (nx + 1), 1.3 / (ny + 1)
    a = np.exp(W.grf_2d(ny + 2, nx + 2, 0.1, 1.0, hx, seed=3))
    f = np.stack([W.rhs_2d_modes(nx, ny, 8, 0.1, 40 + b) for b in range(2)])
    x0 = np.stack([W.rhs_random((ny, nx), 50 + b) for b in range(2)])
    kw = dict(tile=tile, s=s, overlap=ov)
    for lds in (False, True):
        U = dev(x0)
        hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, rel_tol=0.0, max_cycles=3, lds_kernel=lds, **kw)
        got = host(U)
        for b in range(2):
            want = orc.vc_solve_2d(a, f[b], x0[b], hx, hy, tol=0.0, max_cycles=3, **kw)[0]
            assert np.array_equal(got[b], want), f"lds={lds} b={b} fixed cycles"
    U = dev(x0)
    infos = hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, rel_tol=1e-7, **kw)
    got = host(U)
    for b in range(2):
        xo, co, relo, _ = orc.vc_solve_2d(a, f[b], x0[b], hx, hy, tol=1e-7, **kw)
        say(f"vc ragged {tile} s={s} b={b}: gpu cycles {infos[b].cycles}, oracle {co}")
        assert infos[b].cycles == co
        assert np.array_equal(got[b], xo)
        assert abs(infos[b].rel_residual - relo) <= 1e-9 * relo


def test_vc_classical_and_tolerance_match_oracle(orc, prob):
    nx, ny, hx, hy, a, f = prob
    U = torch.zeros_like(dev(f))
    hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, method="global", rel_tol=0.0, max_cycles=17)
    for b in range(f.shape[0]):
        want = orc.vc_solve_2d(a, f[b], np.zeros((ny, nx)), hx, hy, method=orc.CLASSICAL, tol=0.0,
                               max_cycles=17)[0]
        assert np.array_equal(host(U)[b], want)
    U.zero_()
    infos = hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, tile=(32, 32), s=8, overlap=(14, 14),
                           rel_tol=1e-8)
    for b in range(f.shape[0]):
        xo, co, relo, _ = orc.vc_solve_2d(a, f[b], np.zeros((ny, nx)), hx, hy, tile=(32, 32), s=8,
                                          overlap=(14, 14), tol=1e-8)
        say(f"vc solve b={b}: gpu cycles {infos[b].cycles}, oracle {co}")
        assert infos[b].cycles == co
        assert np.array_equal(host(U)[b], xo)
        assert abs(infos[b].rel_residual - relo) <= 1e-9 * relo


def test_vc_batch_equals_single_rhs_solves(prob):
    """Several right-hand sides run through the batched engine; each must end
    where its own single-right-hand-side solve ends: same iterate bit for
    bit, same cycle count, also when some stop at max_cycles."""
    nx, ny, hx, hy, a, f = prob
    opts = dict(hx=hx, hy=hy, tile=(16, 32), s=6, overlap=(10, 10))
    for tol, cap in ((1e-9, 1_000_000), (1e-9, 40)):
        U = torch.zeros_like(dev(f))
        infos = hj.solve_vc_2d(dev(a), dev(f), U, rel_tol=tol, max_cycles=cap, allow_not_converged=True, **opts)
        for b in range(f.shape[0]):
            Ub = torch.zeros_like(dev(f[b:b + 1]))
            one = hj.solve_vc_2d(dev(a), dev(f[b:b + 1]), Ub, rel_tol=tol, max_cycles=cap,
                                 allow_not_converged=True, **opts)[0]
            say(f"vc batch b={b} cap={cap}: batched {infos[b].cycles} single {one.cycles}")
            assert infos[b].cycles == one.cycles <= cap
            assert np.array_equal(host(U)[b], host(Ub)[0])
            assert abs(infos[b].rel_residual - one.rel_residual) <= 1e-12 * one.rel_residual
            assert (infos[b].rel_residual <= tol) == (one.rel_residual <= tol)


def test_vc_gradient_matches_oracle_formula(orc, prob):
    nx, ny, hx, hy, a, f = prob
    u = np.stack([W.rhs_random((ny, nx), 20 + b) for b in range(3)])
    lam = np.stack([W.rhs_random((ny, nx), 30 + b) for b in range(3)])
    g = host(hj.vc_grad_a(dev(a), dev(u), dev(lam), hx=hx, hy=hy))
    want = sum(orc.vc_grad_a_2d(u[b], lam[b], hx, hy) for b in range(3))
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def test_adjoint_solve_and_autograd_against_finite_differences(orc):
    ny, nx = 20, 24
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    a0 = np.exp(W.grf_2d(ny + 2, nx + 2, 0.2, 1.0, hx, seed=11))
    f0 = np.stack([W.rhs_2d_modes(nx, ny, 6, 0.0, s) for s in range(2)])
    t = np.stack([W.smooth_modes_2d(nx, 3, 3, s)[:ny, :] for s in range(2)]) * 1e-3
    opts = dict(hx=hx, hy=hy, tile=(16, 16), s=6, overlap=(10, 10), rel_tol=1e-13)
    T = dev(t)

    def loss_of(A, F):
        return torch.mean((hj.diffusion_solve(F, A, **opts) - T) ** 2)

    A = dev(a0).requires_grad_(True)
    F = dev(f0).requires_grad_(True)
    L = loss_of(A, F)
    L.backward()
    ga, gf = host(A.grad), host(F.grad)

    # against the oracle: same solves on the CPU, adjoint formula for dL/da
    us = [orc.vc_solve_2d(a0, f0[b], np.zeros((ny, nx)), hx, hy, tile=(16, 16), s=6, overlap=(10, 10),
                          tol=1e-13)[0] for b in range(2)]
    n = t.size
    lams = [orc.vc_solve_2d(a0, 2 * (us[b] - t[b]) / n, np.zeros((ny, nx)), hx, hy, tile=(16, 16), s=6,
                            overlap=(10, 10), tol=1e-13)[0] for b in range(2)]
    want_ga = sum(orc.vc_grad_a_2d(us[b], lams[b], hx, hy) for b in range(2))
    assert np.max(np.abs(ga - want_ga)) <= 1e-8 * np.max(np.abs(want_ga))
    assert np.max(np.abs(gf - np.stack(lams))) <= 1e-8 * np.max(np.abs(gf))

    # central finite differences (eps = 1e-6, FP64) of the GPU forward solve
    rng = np.random.default_rng(3)
    eps = 1e-6
    with torch.no_grad():
        for _ in range(8):
            r, q = rng.integers(0, ny + 2), rng.integers(0, nx + 2)
            Ap, Am = dev(a0), dev(a0)
            Ap[r, q] += eps
            Am[r, q] -= eps
            fd = (loss_of(Ap, dev(f0)) - loss_of(Am, dev(f0))).item() / (2 * eps)
            say(f"dL/da[{r},{q}]: autograd {ga[r, q]:.6e} fd {fd:.6e}")
            assert abs(fd - ga[r, q]) <= 1e-4 * np.max(np.abs(ga)) + 1e-6 * abs(ga[r, q])
        for _ in range(4):
            b, r, q = rng.integers(0, 2), rng.integers(0, ny), rng.integers(0, nx)
            Fp, Fm = dev(f0), dev(f0)
            Fp[b, r, q] += eps
            Fm[b, r, q] -= eps
            fd = (loss_of(dev(a0), Fp) - loss_of(dev(a0), Fm)).item() / (2 * eps)
            assert abs(fd - gf[b, r, q]) <= 1e-4 * np.max(np.abs(gf))


@pytest.mark.parametrize("mode", ["fixed", "tol"])
def test_solve_adjoint_c_abi_pitched_batch(orc, mode):
    """hj_solve_adjoint called through the C ABI on a batch of 3 right-hand
    sides in pitched storage: f/u/lam rows of ld > nx, a batch stride beyond
    ny * ld, coefficient rows of lda > nx + 2 and gradient rows of
    ld_grad > nx + 2, starting from a nonzero guess.  lam equals the oracle's
    solve of dL/du bit for bit (fixed cycles; to tolerance also the cycle
    counts), dL/da equals the oracle's face-product gradient summed over the
    batch within 1e-12, and no padding element is written (NaN padding in the
    inputs would also show any read of it in the results)."""
    ny, nx, B = 40, 56, 3
    ld, lda, ldg = nx + 5, nx + 2 + 3, nx + 2 + 6
    bstride = ny * ld + 37
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    a = np.exp(W.grf_2d(ny + 2, nx + 2, 0.15, 1.0, hx, seed=5))
    u = [W.rhs_random((ny, nx), 40 + b) for b in range(B)]
    dl = [W.rhs_2d_modes(nx, ny, 6, 0.1, 50 + b) for b in range(B)]
    lam0 = [W.rhs_random((ny, nx), 60 + b) * 1e-3 for b in range(B)]

    def flat(arrs, fill):
        buf = np.full(B * bstride, fill)
        for b, arr in enumerate(arrs):
            buf[b * bstride: b * bstride + ny * ld].reshape(ny, ld)[:, :nx] = arr
        return buf

    def unflat(buf):
        return [buf[b * bstride: b * bstride + ny * ld].reshape(ny, ld)[:, :nx] for b in range(B)]

    A = np.full((ny + 2, lda), np.nan)
    A[:, :nx + 2] = a
    dA, dU, dDL = dev(A), dev(flat(u, np.nan)), dev(flat(dl, np.nan))
    LAM = dev(flat(lam0, -7.0))
    G = dev(np.full((ny + 2, ldg), -9.0))
    kw = dict(tile=(32, 16), s=5, overlap=(8, 6))
    tol, cycles = (0.0, 7) if mode == "fixed" else (1e-9, 1_000_000)

    pr = hj.VCProblem()
    pr.nx, pr.ny, pr.ld, pr.lda, pr.hx, pr.hy = nx, ny, ld, lda, hx, hy
    pr.a, pr.batch, pr.flags, pr.batch_stride = dA.data_ptr(), B, 0, bstride
    d = hj.AdjointDesc()
    d.prob = pr
    d.u, d.dl_du, d.lam, d.dl_da, d.ld_grad = dU.data_ptr(), dDL.data_ptr(), LAM.data_ptr(), G.data_ptr(), ldg
    d.params = hj.make_params(kw["tile"], kw["s"], "hierarchical", tol, cycles, 0, kw["overlap"])
    infos = (hj._Info * B)()
    torch.cuda.synchronize()
    st = hj.load().hj_solve_adjoint(ctypes.byref(d), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    infos)
    assert st == hj.HJ_OK, hj.last_error()
    lam_buf = host(LAM)
    lams = unflat(lam_buf)
    for b in range(B):
        xo, co, relo, _ = orc.vc_solve_2d(a, dl[b], lam0[b], hx, hy, tile=kw["tile"], s=kw["s"],
                                          overlap=kw["overlap"], tol=tol, max_cycles=cycles)
        say(f"adjoint {mode} b={b}: gpu cycles {infos[b].cycles}, oracle {co}")
        assert np.array_equal(lams[b], xo), f"batch {b}"
        if mode == "tol":
            assert infos[b].cycles == co and abs(infos[b].rel_residual - relo) <= 1e-9 * relo
    # padding of lam untouched
    mask = np.ones(B * bstride, bool)
    for b in range(B):
        mask[b * bstride: b * bstride + ny * ld].reshape(ny, ld)[:, :nx] = False
    assert np.all(lam_buf[mask] == -7.0)
    g = host(G)
    want = sum(orc.vc_grad_a_2d(u[b], lams[b], hx, hy) for b in range(B))
    assert np.all(g[:, nx + 2:] == -9.0)
    assert np.max(np.abs(g[:, :nx + 2] - want)) <= 1e-12 * np.max(np.abs(want))


def test_solve_adjoint_binding_without_gradient(orc, prob):
    """The binding's solve_adjoint with grad_a=False passes NULL dl_da: lam is
    the adjoint solve alone and no gradient is formed."""
    nx, ny, hx, hy, a, f = prob
    Lam = torch.zeros_like(dev(f))
    infos, g = hj.solve_adjoint(dev(a), None, dev(f), Lam, hx=hx, hy=hy, tile=(32, 32), s=8, overlap=(14, 14),
                                rel_tol=0.0, max_cycles=4, grad_a=False)
    assert g is None and len(infos) == f.shape[0]
    for b in range(f.shape[0]):
        want = orc.vc_solve_2d(a, f[b], np.zeros((ny, nx)), hx, hy, tile=(32, 32), s=8, overlap=(14, 14),
                               tol=0.0, max_cycles=4)[0]
        assert np.array_equal(host(Lam)[b], want)


def test_vc_config_size_forward_and_adjoint_match_oracle(orc):
    """The differentiable configuration at its own size: 1024 x 1024,
    a = exp(g) (squared-exponential field, length 0.05, variance 1), 16
    right-hand sides through the batched engine.  Three fixed cycles of the
    forward solve (64 x 32 tiles, s = 8, overlap 14) equal the oracle's per
    right-hand side bit for bit; the adjoint solve through hj_solve_adjoint
    on dL/du = 2 (u - t) / N from those states equals the oracle's solve of
    the same right-hand sides bit for bit, and dL/da equals the oracle's
    face-product gradient summed over the batch within 1e-12."""
    n, B, K = 1024, 16, 3
    h = 1.0 / (n + 1)
    kw = dict(tile=(64, 32), s=8, overlap=(14, 14))
    a = W.diffusion_coefficient(n, 0.05, 1.0, 7)
    f = np.stack([W.rhs_2d_modes(n, n, 8, 0.0, b) for b in range(B)])
    A, F = dev(a), dev(f)
    U = torch.zeros_like(F)
    hj.solve_vc_2d(A, F, U, h, rel_tol=0.0, max_cycles=K, **kw)
    u = host(U)
    for b in range(B):
        want = orc.vc_solve_2d(a, f[b], np.zeros((n, n)), h, h, tol=0.0, max_cycles=K, **kw)[0]
        assert np.array_equal(u[b], want), f"forward, right-hand side {b}"
    t = np.stack([W.smooth_modes_2d(n, 3, 3, 100 + b) for b in range(B)]) * 1e-3
    dl = 2.0 * (u - t) / u.size
    LAM = torch.zeros_like(F)
    infos, G = hj.solve_adjoint(A, U, dev(dl), LAM, h, rel_tol=0.0, max_cycles=K, **kw)
    lam = host(LAM)
    assert len(infos) == B and all(i.cycles == K for i in infos)
    for b in range(B):
        want = orc.vc_solve_2d(a, dl[b], np.zeros((n, n)), h, h, tol=0.0, max_cycles=K, **kw)[0]
        assert np.array_equal(lam[b], want), f"adjoint, right-hand side {b}"
    want_g = sum(orc.vc_grad_a_2d(u[b], lam[b], h, h) for b in range(B))
    g = host(G)
    err = np.max(np.abs(g - want_g)) / np.max(np.abs(want_g))
    say(f"1024^2 x 16: dL/da max difference {err:.2e} of the largest entry")
    assert err <= 1e-12
