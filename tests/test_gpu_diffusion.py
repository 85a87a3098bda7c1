"""GPU parity for variable-coefficient diffusion -div(a grad u) = f and its
adjoint: forward iterates and cycles-to-tolerance against the CPU oracle, the
gradient with respect to a against the oracle's face-product formula (itself
pinned by finite differences of direct solves), and torch autograd through the
adjoint solve against central finite differences."""
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


@pytest.mark.parametrize("tile,s,ov", [((32, 32), 8, (0, 0)), ((16, 16), 4, (6, 6)), ((64, 16), 3, (2, 2))])
def test_vc_fixed_cycles_match_oracle(orc, prob, tile, s, ov):
    nx, ny, hx, hy, a, f = prob
    U = torch.zeros_like(dev(f))
    hj.solve_vc_2d(dev(a), dev(f), U, hx=hx, hy=hy, tile=tile, s=s, overlap=ov, rel_tol=0.0, max_cycles=5)
    got = host(U)
    for b in range(f.shape[0]):
        want = orc.vc_solve_2d(a, f[b], np.zeros((ny, nx)), hx, hy, tile=tile, s=s, overlap=ov,
                               tol=0.0, max_cycles=5)[0]
        assert np.array_equal(got[b], want), f"batch {b}"


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
