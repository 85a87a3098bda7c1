"""Several host threads calling the library at once on one device, each on a
stream of its own: the library serialises calls per device around its shared
scratch, so every solve must return what the same solve returns alone (the
same iterate bit for bit, the same cycle count and residual).  ctypes drops
the GIL around each foreign call, so the calls really overlap."""
import threading

import numpy as np
import pytest

from paper_2006_16465_amd import hj
from paper_2006_16465_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve(kind, f):
    x = torch.zeros_like(f)
    if kind == "2d":
        info = hj.solve_2d(f, x, W.grid_h(f.shape[1]), tile=(64, 32), s=8, overlap=(14, 14), rel_tol=1e-8)
    elif kind == "2d_noalloc":
        info = hj.solve_2d_noalloc(f, x, W.grid_h(f.shape[1]), tile=(32, 32), s=6, overlap=(10, 10),
                                   rel_tol=1e-7)
    else:
        info = hj.solve_1d(f, x, W.grid_h(f.shape[0]), tile=128, s=16, overlap=30, rel_tol=1e-8,
                           launch_per_cycle=True)
    return x, info


def test_concurrent_calls_from_several_threads_match_serial_calls():
    problems = [
        ("2d", torch.from_numpy(W.rhs_2d_modes(256, 192, 8, 0.0, 0)).cuda()),
        ("2d", torch.from_numpy(W.rhs_2d_modes(320, 160, 8, 0.0, 1)).cuda()),
        ("2d_noalloc", torch.from_numpy(W.rhs_2d_modes(200, 256, 8, 0.0, 2)).cuda()),
        ("1d", torch.from_numpy(W.rhs_1d_modes(3000, 8, 3)).cuda()),
    ]
    want = []
    for kind, f in problems:
        x, info = _solve(kind, f)
        torch.cuda.synchronize()
        want.append((x.cpu().numpy(), info.cycles, info.rel_residual))
        print(f"serial {kind} {tuple(f.shape)}: {info.cycles} cycles", flush=True)

    reps = 4
    got = [[None] * reps for _ in problems]
    errors = []

    def worker(i):
        try:
            kind, f = problems[i]
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                for r in range(reps):
                    x, info = _solve(kind, f)
                    stream.synchronize()
                    got[i][r] = (x.cpu().numpy(), info.cycles, info.rel_residual)
        except Exception as e:  # reported below, in the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(len(problems))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in threads), "a worker did not finish"
    assert not errors, errors
    for i, (kind, _) in enumerate(problems):
        for r in range(reps):
            x, cycles, rel = got[i][r]
            assert np.array_equal(x, want[i][0]), f"{kind} problem {i}, repetition {r}"
            assert cycles == want[i][1] and rel == want[i][2], (kind, i, r, cycles, want[i][1])
