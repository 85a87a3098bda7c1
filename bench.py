"""Time-to-tolerance benchmark: hierarchical vs global-memory Jacobi on the
2D 5-point Poisson problem, 4096 x 4096 interior points, FP64, to relative
residual 1e-6, on one MI355X.

One step = solving the five seeded right-hand sides (8 random separable sine
modes each, seeds 0-4) from x0 = 0, one after another, with inputs already
resident in HBM.  `value` is the mean time to tolerance per problem.

Default parameters: 64 x 128 tiles, s = 16 sub-iterations, overlap 22 points
in x and y: the shape hj_autotune_solve picks on seed 5, a right-hand side of
the same recipe that is not timed.  With overlap 2s - 2 (the exact regime) no
owned point is reached by the frozen halo within s sweeps and a cycle is
exactly s classical sweeps; at s = 16, o = 22 the nearest owned points sit
four points inside its reach, where the halo's weight after s sweeps is
4.7e-6 (halo_leak below), and every seed needs the exact regime's cycle
count ceil(classical sweeps / s).  The exact-regime shape of the earlier
default (s = 12, o = 22) is timed beside it (`exact_regime`; the
mixed-precision rows use it too), as are the paper's own setting (32 x 32,
s = 16, no overlap), the global-memory baseline, the 512 x 512 experiment of
Sec. 4.2 (32 x 32 tiles, s in {1, 4, 8, 16, 32}), the batched,
variable-coefficient, 1D and paper-replica rows.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--s 16] [--tile 64 128]
                    [--overlap 22 22] [--seeds 0 1 2 3 4] [--no-cpu] [--no-global]
                    [--no-paper-config] [--no-c2] ...

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = [os.path.join(ROOT, "paper_2006_16465_amd", "csrc", name)
              for name in ("hj_kernels.hip", "hj_tiles.h", "hj_device.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cycle_bytes_per_launch(n, tile, overlap, esize=8):
    """Algorithmic HBM bytes of one hierarchical cycle launch: every tile reads
    its interior plus the edge halo ((tx+2)(ty+2) - 4 points of x), the f
    values of its interior, and writes its owned points of x."""
    from paper_2006_16465_amd import hj
    tx, ty = tile
    ntx = hj.axis_tiles(n, tx, overlap[0])
    nty = hj.axis_tiles(n, ty, overlap[1])
    ex, ey = min(tx, n), min(ty, n)
    per_tile = ((ex + 2) * (ey + 2) - 4) + ex * ey
    return esize * (ntx * nty * per_tile + n * n)


def vc_cycle_bytes(nx, ny, tile, overlap):
    """Algorithmic HBM bytes of one variable-coefficient cycle (FP64): every
    tile reads x over its interior and edge halo, a at the same nodes (the
    face weights of its points), f over its interior, and writes its owned
    points."""
    from paper_2006_16465_amd import hj
    tx, ty = tile
    nt = hj.axis_tiles(nx, tx, overlap[0]) * hj.axis_tiles(ny, ty, overlap[1])
    ex, ey = min(tx, nx), min(ty, ny)
    halo = (ex + 2) * (ey + 2) - 4
    return 8 * (nt * (2 * halo + ex * ey) + nx * ny)


def sweep_bytes_per_launch(n, esize=8):
    """Algorithmic HBM bytes of one global sweep: read x and f, write x."""
    return 3 * esize * n * n


def cycle_kernel_name(tile, n):
    """Name of the cycle kernel the library runs for this tile on an n x n
    grid: register-resident tiles of C = tx/16 columns and R rows per lane over
    W wavefronts (R = ty/4 up to 64 x 32; 4 rows, 8 at tx = 32, above), else
    the LDS kernel."""
    tx, ty = tile
    if tx in (32, 64, 128) and ty in (16, 32, 64, 128) and n >= max(tile):
        r = ty // 4 if (tx <= 64 and ty <= 32) else (8 if tx == 32 else 4)
        return f"k_cycle2d_reg<double,{tx // 16},{r},{ty // (4 * r)},true,true>"
    return f"k_cycle2d<double,{tx},{ty},true,true>"


LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12  # 256 CUs x 128 B per clock x 2.4 GHz


def cycle_lds_bytes_per_launch(n, tile, overlap, s, esize=8):
    """LDS bytes one launch of the register-resident cycle moves: every sweep,
    each thread writes the first and last rows of its C columns (its row
    group's interface rows) and reads the two neighbouring groups' rows (the
    frozen halo rows at the tile edge): 4 C values per thread and sweep.
    None for the LDS ping-pong kernel."""
    from paper_2006_16465_amd import hj
    tx, ty = tile
    if not cycle_kernel_name(tile, n).startswith("k_cycle2d_reg"):
        return None
    c = tx // 16
    r = ty // 4 if (tx <= 64 and ty <= 32) else (8 if tx == 32 else 4)
    threads = 64 * (ty // (4 * r))
    tiles = hj.axis_tiles(n, tx, overlap[0]) * hj.axis_tiles(n, ty, overlap[1])
    return tiles * threads * s * 4 * c * esize


def kernel_source_hash():
    """Hash of the sources that define the cycle and sweep kernels."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"{name}.counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--tile", type=int, nargs=2, default=[64, 128])
    ap.add_argument("--s", type=int, default=16)
    ap.add_argument("--overlap", type=int, nargs=2, default=[22, 22])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2, 3, 4])
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=0, help="0: adaptive polling")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-global", action="store_true", help="skip the global-memory baseline")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip the paper-setting row (32 x 32 tiles, s = 16, no overlap)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-cycles + FP64-refinement rows (to 1e-10)")
    ap.add_argument("--mixed-tol", type=float, default=1e-10)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched rows (512 2D + 128 1D problems)")
    ap.add_argument("--batch-cycles", type=int, default=24,
                    help="fixed cycles of the batched-vs-one-call-per-problem comparison")
    ap.add_argument("--batch-cap", type=int, default=2000,
                    help="cycle cap of the batched solve to --batch-tol")
    ap.add_argument("--batch-tol", type=float, default=1e-8)
    ap.add_argument("--no-diffusion", action="store_true",
                    help="skip the variable-coefficient / adjoint rows")
    ap.add_argument("--no-1d", action="store_true", help="skip the 1D rows")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact-regime row (s = --exact-s, overlap 2s - 2)")
    ap.add_argument("--exact-s", type=int, default=12,
                    help="s of the exact-regime row and of the mixed-precision rows")
    ap.add_argument("--no-tuned", action="store_true",
                    help="skip the row with the shape hj_autotune_solve picks on an independent seed")
    ap.add_argument("--no-c2", action="store_true",
                    help="skip the 512^2 rows (Sec. 4.2 experiment: 32 x 32 tiles, s in {1, 4, 8, 16, 32})")
    ap.add_argument("--no-replica", action="store_true",
                    help="skip the rows on the paper's own experiment shapes (b = 1, x0 = 1, 1e-4)")
    ap.add_argument("--inner-tol", type=float, default=1e-6)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method runs on a single device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_16465_amd import hj
    from paper_2006_16465_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    hj.load()
    dev = torch.device("cuda:0")
    n = args.n
    h = W.grid_h(n)
    tile, ov, s = tuple(args.tile), tuple(args.overlap), args.s

    log(f"generating {len(args.seeds)} right-hand sides {n}x{n} ...")
    fs = [torch.from_numpy(W.rhs_2d_modes(n, n, 8, 0.0, sd)).to(dev) for sd in args.seeds]
    xs = [torch.zeros_like(fs[0]) for _ in fs]
    stream = torch.cuda.current_stream(dev)

    def run_all(method, tile=tile, s=s, ov=ov):
        """Solve every seed once; returns per-seed (ms by events, info)."""
        out = []
        for f, x in zip(fs, xs):
            x.zero_()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            info = hj.solve_2d(f, x, h, tile=tile, s=s, overlap=ov, method=method,
                               rel_tol=args.tol, check_every=args.check_every)
            e1.record(stream)
            e1.synchronize()
            out.append((e0.elapsed_time(e1), info))
        return out

    def timed(method, steps, warmup, **kw):
        for _ in range(warmup):
            run_all(method, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per = [run_all(method, **kw) for _ in range(steps)]
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        return wall_ms, per

    log(f"hierarchical: tile={tile} s={s} overlap={ov}, {args.warmup} warmup + {args.steps} steps")
    wall_h, per_h = timed("hierarchical", args.steps, args.warmup)
    ms_per_step = wall_h / args.steps
    nprob = len(fs)
    cycles_h = [info.cycles for _, info in per_h[0]]
    ev_ms_h = np.array([[ms for ms, _ in step] for step in per_h])  # steps x seeds
    seed_ms_h = np.median(ev_ms_h, axis=0)

    # dominant kernel: the hierarchical cycle with fused residual.  A solve
    # to tolerance ends with a partial launch (the one whose first workgroup
    # reaches the verdict: later workgroups return) and early-exit launches,
    # so the launch duration is measured on solves that never converge
    # (rel_tol far below reach): every launch is a whole cycle of the same
    # kernel.  Two such solves of K1 < K2 cycles on the same right-hand side,
    # timed with HIP events on the solve stream; their difference over K2 - K1
    # removes the solve's fixed cost (the residual and judge launches that
    # close it).
    bpl = cycle_bytes_per_launch(n, tile, ov)
    avg_launch_s = full_launch_seconds(torch, hj, fs[-1], xs[-1], h, tile, s, ov, stream)
    achieved = bpl / avg_launch_s / 1e9
    copy_gbs = copy_ceiling_gbs(torch, stream)
    kname = f"cycle2d_f64_t{tile[0]}x{tile[1]}_s{s}_o{ov[0]}x{ov[1]}_n{n}"
    traffic = load_traffic(kname)
    kern = cycle_kernel_name(tile, n)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": kern,
        "algorithmic_bytes_per_launch": bpl,
        "avg_launch_us": round(avg_launch_s * 1e6, 2),
        "avg_launch_from": "whole launches of the same kernel (solves that do not converge, 8 and 32 cycles)",
        "copy_ceiling_gbs": round(copy_gbs, 1),
        "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
        "launches_per_step": sum(c + 2 for c in cycles_h),
    }
    if traffic:
        roofline["traffic_gbs"] = round(traffic / avg_launch_s / 1e9, 1)
    lds = cycle_lds_bytes_per_launch(n, tile, ov, s)
    if lds is not None:
        lds_tbs = lds / avg_launch_s / 1e12
        roofline["lds"] = {"bytes_per_launch": lds, "achieved_tbs": round(lds_tbs, 2),
                           "peak_tbs": round(LDS_PEAK_TBS, 2), "frac": round(lds_tbs / LDS_PEAK_TBS, 4)}
    ntiles = hj.axis_tiles(n, tile[0], ov[0]) * hj.axis_tiles(n, tile[1], ov[1])
    roofline["point_sweeps_per_s"] = {
        "owned_g": round(n * n * s / avg_launch_s / 1e9, 1),
        "computed_g": round(ntiles * min(tile[0], n) * min(tile[1], n) * s / avg_launch_s / 1e9, 1)}

    extra = {
        "cycles_per_seed": dict(zip(map(str, args.seeds), cycles_h)),
        "ms_per_seed": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in seed_ms_h])),
        "ms_per_seed_min": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in ev_ms_h.min(axis=0)])),
        "ms_per_seed_max": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in ev_ms_h.max(axis=0)])),
        "rel_residual_per_seed": [info.rel_residual for _, info in per_h[0]],
        "run": run_info(torch),
    }

    glob = None
    if not args.no_global:
        log("global-memory Jacobi baseline")
        wall_g, per_g = timed("global", max(1, args.steps), args.warmup)
        ev_ms_g = np.array([[ms for ms, _ in step] for step in per_g])
        sweeps_g = [info.cycles for _, info in per_g[0]]
        seed_ms_g = np.median(ev_ms_g, axis=0)
        glaunch = sum(c + 2 for c in sweeps_g)
        g_avg = float(ev_ms_g.sum(axis=1).mean()) * 1e-3 / glaunch
        glob = {
            "ms_per_problem": round(wall_g / max(1, args.steps) / nprob, 3),
            "sweeps_per_seed": dict(zip(map(str, args.seeds), sweeps_g)),
            "ms_per_seed": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in seed_ms_g])),
            "sweep_kernel_gbs": round(sweep_bytes_per_launch(n) / g_avg / 1e9, 1),
            "avg_launch_us": round(g_avg * 1e6, 2),
        }
        extra["global_baseline"] = glob
        extra["speedup_vs_global"] = round(glob["ms_per_problem"] / (ms_per_step / nprob), 3)
        extra["speedup_vs_global_per_seed"] = {
            k: round(glob["ms_per_seed"][k] / extra["ms_per_seed"][k], 3) for k in glob["ms_per_seed"]}

    if not args.no_paper_config:
        log("paper setting: 32 x 32 tiles, s = 16, no overlap")
        wall_p, per_p = timed("hierarchical", args.steps, args.warmup, tile=(32, 32), s=16, ov=(0, 0))
        ev_ms_p = np.array([[ms for ms, _ in step] for step in per_p])
        extra["paper_config"] = {
            "tile": [32, 32], "s": 16, "overlap": [0, 0],
            "ms_per_problem": round(wall_p / args.steps / nprob, 3),
            "cycles_per_seed": dict(zip(map(str, args.seeds), [i.cycles for _, i in per_p[0]])),
            "ms_per_seed": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in np.median(ev_ms_p, axis=0)])),
            "timing": f"{args.warmup} warmup + {args.steps} timed steps, per-seed medians",
        }

    s_x = args.exact_s
    ov_exact = (2 * s_x - 2, 2 * s_x - 2)
    if not args.no_exact and (s_x, ov_exact) != (s, tuple(ov)):
        log(f"exact regime: s = {s_x}, overlap {ov_exact}")
        wall_x, per_x = timed("hierarchical", args.steps, args.warmup, s=s_x, ov=ov_exact)
        ev_ms_x = np.array([[ms for ms, _ in step] for step in per_x])
        t_x = full_launch_seconds(torch, hj, fs[-1], xs[-1], h, tile, s_x, ov_exact, stream)
        b_x = cycle_bytes_per_launch(n, tile, ov_exact)
        extra["exact_regime"] = {
            "tile": list(tile), "s": s_x, "overlap": list(ov_exact), "halo_leak": 0.0,
            "avg_launch_us": round(t_x * 1e6, 2),
            "roofline_frac": round(b_x / t_x / 1e9 / HBM_PEAK_GBS, 4),
            "ms_per_problem": round(wall_x / args.steps / nprob, 3),
            "cycles_per_seed": dict(zip(map(str, args.seeds), [i.cycles for _, i in per_x[0]])),
            "ms_per_seed": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in np.median(ev_ms_x, axis=0)])),
            "headline_speedup_over_it": round(wall_x / wall_h, 3),
        }

    if not args.no_tuned:
        # the right-hand-side tuner run on independent right-hand sides of
        # the same workload (seeds 5-7, not timed here; a shape must reach the
        # tolerance on all three), its shape then solving seeds 0-4 like the
        # headline
        log("shape tuned on seeds 5-7 with hj_autotune_solve, applied to the timed seeds")
        f5 = torch.from_numpy(np.stack([W.rhs_2d_modes(n, n, 8, 0.0, sd) for sd in (5, 6, 7)])).to(dev)
        t0 = time.perf_counter()
        tt, ts, tov, _ = hj.autotune_solve(f5, None, h, trial_tol=args.tol)
        tune_s = time.perf_counter() - t0
        del f5
        wall_t, per_t = timed("hierarchical", args.steps, args.warmup, tile=tt, s=ts, ov=tov)
        extra["tuned_shape"] = {
            "tile": list(tt), "s": ts, "overlap": list(tov), "tuning_s": round(tune_s, 2),
            "tuned_on": "seeds 5, 6, 7 together (hj_autotune_solve, trial solves of each to the same tolerance, "
                        "scored by their sum, inexact overlaps included)",
            "halo_leak": halo_leak(ts, min(tov)),
            "ms_per_problem": round(wall_t / args.steps / nprob, 3),
            "cycles_per_seed": dict(zip(map(str, args.seeds), [i.cycles for _, i in per_t[0]])),
            "ms_per_seed": dict(zip(map(str, args.seeds), [round(float(v), 3) for v in np.median(
                np.array([[ms for ms, _ in step] for step in per_t]), axis=0)])),
        }
        log(f"tuned shape: {extra['tuned_shape']}")
    if not args.no_c2:
        extra["poisson2d_512"] = c2_rows(torch, hj, stream)
    if not args.no_mixed:
        extra["mixed_precision"] = mixed_rows(args, torch, hj, fs, xs, h, tile, s_x, ov_exact, stream)
    if not args.no_batch:
        del fs, xs
        torch.cuda.empty_cache()
        extra["batched"] = batched_rows(args, torch, hj, stream)
    if not args.no_diffusion:
        extra["differentiable"] = diffusion_rows(torch, hj, stream)
    if not args.no_1d:
        extra["poisson1d"] = rows_1d(torch, hj, stream)
    if not args.no_replica:
        extra["paper_replicas"] = replica_rows(torch, hj, stream)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, W, cycles_h, tile, ov, s, seed_ms_h)

    line = {
        "metric": "time to rel. residual 1e-6 (2D 4096^2) + achieved HBM GB/s, hierarchical vs global Jacobi",
        "value": round(ms_per_step / nprob, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"poisson2d_{n}: 2D 5-point Poisson {n}x{n}, Dirichlet 0, f = 8 random separable "
                        f"sine modes (seeds {args.seeds}), x0 = 0, to rel. residual {args.tol:g}; one step "
                        f"= all seeds solved once; value = mean ms per problem",
            "n": n, "tile": list(tile), "s": s, "overlap": list(ov), "halo_leak": halo_leak(s, min(ov)),
            "tol": args.tol,
            "seeds": args.seeds, "method": "hierarchical", "check_every": args.check_every,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


def halo_leak(s, o):
    """Weight of the frozen halo in an owned point after the s sweeps of a
    cycle, at the owned point nearest the tile edge (ceil(o/2) + 1 points
    from the halo column).  A 2D Jacobi sweep averages the four neighbours, so
    an iterate is a random-walk expectation and the stale halo enters with
    the probability that the walk's x-coordinate (a lazy walk: -1, 0, +1 with
    probabilities 1/4, 1/2, 1/4) reaches the halo within s - 1 steps (the
    first sweep reads the halo at its current value).  By the reflection
    principle that is P(X <= -d) + P(X <= -d - 1), X = B(2(s-1), 1/2) - (s-1).
    0 in the exact regime (o >= 2s - 2)."""
    from math import comb
    d, m = -(-o // 2) + 1, s - 1
    if d > m:
        return 0.0
    tail = lambda k: sum(comb(2 * m, j) for j in range(0, m - k + 1)) / 4.0 ** m  # P(X <= -k)
    return float(tail(d) + tail(d + 1))


def full_launch_seconds(torch, hj, f, x, h, tile, s, ov, stream, k1=8, k2=32):
    """Mean duration of one whole launch of the fused-residual cycle kernel:
    (t(k2 cycles) - t(k1 cycles)) / (k2 - k1) over solves whose tolerance is
    out of reach, so no launch returns early."""
    def run(k):
        x.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = hj.solve_2d(f, x, h, tile=tile, s=s, overlap=ov, rel_tol=1e-300, max_cycles=k,
                           allow_not_converged=True)
        e1.record(stream)
        e1.synchronize()
        assert info.cycles == k
        return e0.elapsed_time(e1) * 1e-3
    run(k1)
    t1 = min(run(k1) for _ in range(3))
    t2 = min(run(k2) for _ in range(3))
    return (t2 - t1) / (k2 - k1)


def copy_ceiling_gbs(torch, stream, nbytes=1 << 30):
    """Plain device-to-device copy (torch copy_), bytes read + written per
    second: the practical HBM ceiling the kernels are compared with."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        best = t if best is None else min(best, t)
    del src, dst
    return 2 * nbytes / best / 1e9


def run_info(torch):
    """Where the numbers come from: GPU, ROCm, clocks, host CPU."""
    import glob
    import platform
    info = {"gpu": torch.cuda.get_device_name(0), "torch": torch.__version__, "hip": torch.version.hip,
            "host_threads": len(os.sched_getaffinity(0)), "python": platform.python_version()}
    try:
        info["gcn_arch"] = torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as fh:
                levels = [ln.strip() for ln in fh if ln.strip()]
            mhz = [int(ln.split()[1].rstrip("Mhz").rstrip("MHz")) for ln in levels if "hz" in ln.lower()]
            if mhz:
                info["sclk_max_mhz"] = max(mhz)
                cur = [ln for ln in levels if ln.endswith("*")]
                if cur:
                    info["sclk_at_read_mhz"] = int(cur[0].split()[1].rstrip("Mhz").rstrip("MHz"))
                break
        except (OSError, ValueError, IndexError):
            continue
    try:
        with open("/opt/rocm/.info/version") as fh:
            info["rocm"] = fh.read().strip()
    except OSError:
        pass
    return info


def c2_rows(torch, hj, stream):
    """The 2D experiment of Sec. 4.2 on the 512 x 512 workload: 16 separable
    sine modes plus white noise (standard deviation 0.1), x0 = 0, to 1e-6,
    seeds 0-2; global-memory Jacobi against hierarchical Jacobi with 32 x 32
    tiles and s in {1, 4, 8, 16, 32} without overlap, plus the paper's best
    2D overlap (k = 32, o = 4, Table 4).  One timed solve each (after one
    untimed solve of every setting on seed 0).  Cycle counts are compared
    with the oracle's (tests/golden/c2_poisson2d_512.json, written by the
    oracle) where that file holds them."""
    from paper_2006_16465_amd import workloads as W
    log("poisson2d_512 (Sec. 4.2 experiment): global vs 32 x 32 tiles, s in {1, 4, 8, 16, 32}")
    golden = {}
    gpath = os.path.join(ROOT, "tests", "golden", "c2_poisson2d_512.json")
    if os.path.exists(gpath):
        with open(gpath) as fh:
            for c in json.load(fh)["cases"]:
                golden[(c["seed"], c["method"])] = c["cycles"]
    settings = [("global", dict(method="global"))]
    settings += [(f"s{k}", dict(tile=(32, 32), s=k, overlap=(0, 0))) for k in (1, 4, 8, 16, 32)]
    settings += [("s32_o4", dict(tile=(32, 32), s=32, overlap=(4, 4)))]
    seeds = (0, 1, 2)
    fs = {sd: torch.from_numpy(W.make("poisson2d_512", sd)[0]).cuda() for sd in seeds}
    h = W.grid_h(512)
    x = torch.zeros_like(fs[0])
    out = {"workload": "poisson2d_512: 2D 512x512, f = 16 random separable sine modes + white noise "
                       "(sigma 0.1), x0 = 0, to rel. residual 1e-6, seeds 0-2", "rows": {}}

    def solve(f, kw):
        x.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = hj.solve_2d(f, x, h, rel_tol=1e-6, max_cycles=10_000_000, **kw)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), info

    for name, kw in settings:
        x.zero_()
        hj.solve_2d(fs[0], x, h, rel_tol=0.0, max_cycles=10, **kw)  # untimed: scratch, code objects
        ms, cyc, match = [], [], []
        for sd in seeds:
            t, info = solve(fs[sd], kw)
            ms.append(round(t, 2))
            cyc.append(info.cycles)
            key = (sd, "classical" if name == "global" else name)
            if key in golden:
                match.append(golden[key] == info.cycles)
        row = {"ms_per_seed": ms, "cycles_per_seed": cyc, "ms_per_problem": round(float(np.mean(ms)), 2)}
        if match:
            row["cycles_equal_oracle"] = all(match)
        out["rows"][name] = row
        log(f"poisson2d_512 {name}: {row}")
    g = out["rows"]["global"]["ms_per_problem"]
    out["speedup_vs_global"] = {k: round(g / v["ms_per_problem"], 2) for k, v in out["rows"].items() if k != "global"}
    out["paper_reported"] = {"note": "Table 3 (b = 1, x0 = 1, 1e-4, 1024^2, its own GPU): 2.17 / 3.67 / 3.98 / "
                                     "2.96 at k = 4 / 8 / 16 / 32; Table 4 best overlap k = 32, o = 4: 5.84"}
    return out


def mixed_rows(args, torch, hj, fs, xs, h, tile, s, ov, stream):
    """FP64 hierarchical cycles vs FP32 cycles inside FP64 iterative refinement,
    both to args.mixed_tol on the same right-hand sides (per-seed medians of
    5 interleaved timed calls each).  The FP64 path equals
    the CPU oracle bit for bit (GPU tests); the refined solution's distance to
    it is reported per seed.  Two shapes: the exact-regime shape of the
    headline rows (top-level keys), and the workload's own 64x64 tiles with s
    and overlap from hj_autotune_solve restricted to that tile, tuned on
    right-hand sides the timed seeds do not include (config3_64x64)."""
    from paper_2006_16465_amd import workloads as W

    log(f"mixed precision: FP64 vs FP32 + FP64 refinement to {args.mixed_tol:g}")
    x64 = torch.zeros_like(fs[0])

    def timed_call(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), r

    def rows(tile, s, ov):
        exact = min(ov) >= 2 * s - 2
        out = {"tile": list(tile), "s": s, "overlap": list(ov), "tol": args.mixed_tol,
               "inner_tol": args.inner_tol,
               "switch_tol": (1e5 if exact else 1e4) * args.mixed_tol,
               "switch_rule": "library default: 1e5 tol in the exact regime (overlap >= 2s - 2), else 1e4 tol",
               "fp64_ms": {}, "refined_ms": {},
               "fp64_cycles": {}, "refined_fp64_cycles": {}, "refined_inner_cycles": {}, "refined_outer": {},
               "rel_diff_refined_vs_fp64": {}}
        for sd, f, x in zip(args.seeds, fs, xs):
            # one untimed call of each (scratch warm-up), then 5 interleaved timed
            # calls of each; per-seed medians
            t64s, tmxs = [], []
            for rep in range(6):
                x64.zero_()
                t64, i64 = timed_call(lambda: hj.solve_2d(f, x64, h, tile=tile, s=s, overlap=ov,
                                                          rel_tol=args.mixed_tol))
                x.zero_()
                tmx, imx = timed_call(lambda: hj.solve_2d_refined(
                    f, x, h, tile=tile, s=s, overlap=ov, rel_tol=args.mixed_tol, inner_tol=args.inner_tol))
                if rep > 0:
                    t64s.append(t64)
                    tmxs.append(tmx)
            k = str(sd)
            out["fp64_ms"][k] = round(float(np.median(t64s)), 3)
            out["refined_ms"][k] = round(float(np.median(tmxs)), 3)
            out["fp64_cycles"][k] = i64.cycles
            out["refined_fp64_cycles"][k] = imx.fp64_cycles
            out["refined_inner_cycles"][k] = imx.inner_cycles
            out["refined_outer"][k] = imx.outer
            out["rel_diff_refined_vs_fp64"][k] = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        out["fp64_ms_per_problem"] = round(sum(out["fp64_ms"].values()) / len(fs), 3)
        out["refined_ms_per_problem"] = round(sum(out["refined_ms"].values()) / len(fs), 3)
        out["speedup_refined_vs_fp64"] = round(out["fp64_ms_per_problem"] / out["refined_ms_per_problem"], 3)
        return out

    res = rows(tile, s, ov)
    n = fs[0].shape[0]
    tune_seeds = (5, 6, 7)
    f5 = torch.from_numpy(np.stack([W.rhs_2d_modes(n, n, 8, 0.0, sd) for sd in tune_seeds])).to(fs[0].device)
    t0 = time.perf_counter()
    # trial solves to the row's own tolerance: a near-exact overlap that wins
    # at 1e-6 can stall on the way to 1e-10 (the stale halo's small weight
    # matters more the further the residual has to fall)
    t3, s3, ov3, _ = hj.autotune_solve(f5, None, h, trial_tol=args.mixed_tol, tile=(64, 64))
    tune_s = time.perf_counter() - t0
    del f5
    log(f"mixed precision, 64x64 tiles: tuned s {s3}, overlap {ov3} ({tune_s:.1f} s)")
    res["config3_64x64"] = rows(t3, s3, ov3)
    res["config3_64x64"]["tuned_on"] = (f"seeds {', '.join(map(str, tune_seeds))} together: hj_autotune_solve "
                                        f"with the tile fixed at 64x64, FP64 trial solves to {args.mixed_tol:g}")
    res["config3_64x64"]["tuning_s"] = round(tune_s, 2)
    return res


def batched_rows(args, torch, hj, stream):
    """512 square 2D problems (side log-uniform in [64, 1024]) and 128 1D
    problems (N log-uniform in [1e3, 1e6]), FP64, random-mode right-hand sides
    (workloads.batch_specs).  Shapes from the autotuner.  (1) A fixed number of
    cycles of every problem: one hj_solve_batched call against one
    hj_solve_2d / hj_solve_1d call per problem (same iterates, checked).
    (2) The batched solve to --batch-tol with a cycle cap: a few problems hold
    a mode so smooth that Jacobi needs millions of sweeps, so the cap decides
    how many converge; the same cap is applied to the per-problem calls."""
    from paper_2006_16465_amd import workloads as W
    log("batched: building 512 2D + 128 1D problems")
    specs = W.batch_specs(0)
    table = []
    for spec in specs:
        F = torch.from_numpy(W.batch_rhs(spec)).to("cuda")
        table.append((F, torch.zeros_like(F), 1.0 / (spec[1] + 1)))
    (t2, s2, o2), (t1, s1, o1) = hj.autotune_batch(table)
    log(f"batched: autotuned 2D tile {t2} s {s2} overlap {o2}; 1D tile {t1} s {s1} overlap {o1}")
    shape = dict(tile=t2, s=s2, overlap=o2, tile_1d=t1, s_1d=s1, overlap_1d=o1)
    dof = sum(n * n if d == 2 else n for d, n, _ in specs)
    sweeps_per_cycle = sum((n * n * s2) if d == 2 else (n * s1) for d, n, _ in specs)

    def clear():
        for _, x, _ in table:
            x.zero_()
        torch.cuda.synchronize()

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r = fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), r

    def one_by_one(rel_tol, cap):
        out = []
        for F, X, h in table:
            if F.dim() == 2:
                out.append(hj.solve_2d(F, X, h, tile=t2, s=s2, overlap=o2, rel_tol=rel_tol, max_cycles=cap,
                                       allow_not_converged=True))
            else:
                out.append(hj.solve_1d(F, X, h, tile=t1, s=s1, overlap=o1, rel_tol=rel_tol, max_cycles=cap,
                                       allow_not_converged=True))
        return out

    K = args.batch_cycles
    clear()
    hj.solve_batched(table, rel_tol=0.0, max_cycles=2, **shape)  # warm-up (graph, scratch)
    clear()
    tb, _ = timed(lambda: hj.solve_batched(table, rel_tol=0.0, max_cycles=K, **shape))
    xb = [x.clone() for _, x, _ in table]
    clear()
    one_by_one(0.0, 2)
    clear()
    ts, _ = timed(lambda: one_by_one(0.0, K))
    same = all(torch.equal(a, x) for a, (_, x, _) in zip(xb, table))
    del xb
    log(f"batched: {K} cycles: batched {tb:.1f} ms, one call per problem {ts:.1f} ms, identical {same}")

    C, tol = args.batch_cap, args.batch_tol
    clear()
    tt, infos = timed(lambda: hj.solve_batched(table, rel_tol=tol, max_cycles=C, allow_not_converged=True,
                                               **shape))
    conv = [i for i in infos if i.status == hj.HJ_OK]
    clear()
    tts, infos_s = timed(lambda: one_by_one(tol, C))
    conv_s = sum(1 for i in infos_s if i.status == hj.HJ_OK)
    log(f"batched: to {tol:g} (cap {C} cycles): batched {tt:.1f} ms ({len(conv)} of {len(infos)} converged), "
        f"one call per problem {tts:.1f} ms ({conv_s})")
    clear()
    tr, infos_r = timed(lambda: hj.solve_batched(table, rel_tol=tol, max_cycles=C, refine=True, max_outer=3,
                                                 allow_not_converged=True, **shape))
    conv_r = sum(1 for i in infos_r if i.status == hj.HJ_OK)
    log(f"batched: to {tol:g} with FP32 corrections in FP64 refinement (cap {C} cycles per problem, all phases): "
        f"{tr:.1f} ms ({conv_r} of {len(infos_r)} converged)")
    cyc = np.array([i.cycles for i in conv]) if conv else np.array([0])
    return {
        "workload": "512 square 2D (side log-uniform [64, 1024]) + 128 1D (N log-uniform [1e3, 1e6]) Poisson "
                    "problems, FP64, 8 random sine modes each, x0 = 0 (workloads.batch_specs(0))",
        "dof": int(dof),
        "shapes": {"2d": {"tile": list(t2), "s": s2, "overlap": list(o2)},
                   "1d": {"tile": t1, "s": s1, "overlap": o1}, "by": "autotuner (hj_autotune_batch)"},
        "fixed_cycles": {"cycles": K, "batched_ms": round(tb, 2), "one_call_per_problem_ms": round(ts, 2),
                         "speedup": round(ts / tb, 2), "identical_iterates": bool(same),
                         "batched_gsweeps_per_s": round(sweeps_per_cycle * K / (tb * 1e-3) / 1e9, 1)},
        "to_tol": {"tol": tol, "cycle_cap": C, "batched_ms": round(tt, 2),
                   "one_call_per_problem_ms": round(tts, 2), "converged": len(conv),
                   "converged_one_call_per_problem": conv_s, "problems": len(infos),
                   "cycles_median_converged": float(np.median(cyc)), "cycles_max_converged": int(cyc.max())},
        "to_tol_refined": {"tol": tol, "method": "per problem: FP64 cycles down to min(1e4 tol, tol / 8F) "
                           "(F its predicted FP32 floor), then FP32 corrections inside FP64 refinement "
                           "(hj_solve_batched, HJ_BATCH_REFINE)", "cycle_cap": C,
                           "max_outer": 3, "ms": round(tr, 2), "converged": conv_r, "problems": len(infos_r),
                           "cycles_sum": int(sum(i.cycles for i in infos_r)),
                           "cycles_sum_fp64": int(sum(i.cycles for i in infos))},
    }


def rows_1d(torch, hj, stream):
    """1D Poisson, N = 256 interior points, 8 random sine modes (seeds 0-4),
    x0 = 0, to 1e-6: the paper's setting (32-point tiles, s = 16, no overlap),
    64-point tiles with s = 8 and overlap 14 (a cycle = 8 classical sweeps;
    the five tiles fit one workgroup, which runs every cycle in one launch),
    the same shape with one launch per cycle, and classical Jacobi both ways:
    inside one workgroup (the library's default for a grid this small: s = 1
    cycles without overlap are classical sweeps) and one launch per sweep.
    Mean ms per problem (median of 5 repeats).  Speedups are quoted against
    the classical solve with the same launch treatment."""
    from paper_2006_16465_amd import workloads as W
    n = 256
    h = W.grid_h(n)
    fs = [torch.from_numpy(W.rhs_1d_modes(n, 8, sd)).cuda() for sd in range(5)]
    x = torch.zeros_like(fs[0])
    out = {"workload": "poisson1d_n256: -u'' = f, N = 256, f = 8 random sine modes (seeds 0-4), x0 = 0, to 1e-6"}
    for name, kw in (("paper_t32_s16", dict(tile=32, s=16, overlap=0)),
                     ("overlap_t64_s8_o14", dict(tile=64, s=8, overlap=14)),
                     ("overlap_t64_s8_o14_launch_per_cycle", dict(tile=64, s=8, overlap=14, launch_per_cycle=True)),
                     ("global_one_workgroup", dict(method="global")),
                     ("global_launch_per_sweep", dict(method="global", launch_per_cycle=True))):
        ms, cyc = [], []
        for f in fs:
            reps = []
            for _ in range(5):
                x.zero_()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                info = hj.solve_1d(f, x, h, rel_tol=1e-6, **kw)
                e1.record(stream)
                e1.synchronize()
                reps.append(e0.elapsed_time(e1))
            ms.append(float(np.median(reps)))
            cyc.append(info.cycles)
        out[name] = {"ms_per_problem": round(float(np.mean(ms)), 3), "cycles_per_seed": cyc}
    assert out["global_one_workgroup"]["cycles_per_seed"] == out["global_launch_per_sweep"]["cycles_per_seed"]
    g1 = out["global_one_workgroup"]["ms_per_problem"]
    gl = out["global_launch_per_sweep"]["ms_per_problem"]
    out["speedup_overlap_one_workgroup_vs_global_one_workgroup"] = round(g1 / out["overlap_t64_s8_o14"]["ms_per_problem"], 2)
    out["speedup_overlap_launch_per_cycle_vs_global_launch_per_sweep"] = round(
        gl / out["overlap_t64_s8_o14_launch_per_cycle"]["ms_per_problem"], 2)
    out["speedup_paper_setting_vs_global_launch_per_sweep"] = round(gl / out["paper_t32_s16"]["ms_per_problem"], 2)
    log(f"1d: {out}")
    return out


def replica_rows(torch, hj, stream):
    """The paper's own experiment shapes (b = 1, x0 = 1, relative residual
    1e-4): (R1) 1024 independent 1D systems of N = 1024 side by side, one
    hj_solve_batched call each way, every step one launch over all copies;
    (R2) one 2D 1024^2 system.  Global-memory Jacobi (1D: cycles with s = 1,
    which are classical sweeps; 2D: the global sweep kernel) against the
    paper's setting (32-point / 32x32 tiles, s = 16, no overlap) and an
    overlapped shape (a cycle = s classical sweeps).  The paper's ~8x (1D)
    and ~6x (2D) were measured on its own GPU: context, not a target."""
    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, r

    out = {}
    n, copies = 1024, 1024
    h = 1.0 / (n + 1)
    F = torch.ones(n, dtype=torch.float64, device="cuda")
    xs = [torch.empty_like(F) for _ in range(copies)]
    table = [(F, x, h) for x in xs]
    r1 = {"workload": "1024 copies of 1D -u'' = 1, N = 1024, x0 = 1, to 1e-4 (one batched call)"}
    for name, kw in (("global", dict(tile_1d=256, s_1d=1, overlap_1d=0)),
                     ("global_one_workgroup", dict(tile_1d=256, s_1d=1, overlap_1d=0, one_workgroup_1d=True)),
                     ("paper_t32_s16", dict(tile_1d=32, s_1d=16, overlap_1d=0)),
                     ("paper_t32_s16_o4", dict(tile_1d=32, s_1d=16, overlap_1d=4)),
                     ("overlap_t256_s32_o62", dict(tile_1d=256, s_1d=32, overlap_1d=62)),
                     ("overlap_t256_s32_o62_one_workgroup",
                      dict(tile_1d=256, s_1d=32, overlap_1d=62, one_workgroup_1d=True))):
        for x in xs:
            x.fill_(1.0)
        ms, infos = timed(lambda: hj.solve_batched(table, rel_tol=1e-4, max_cycles=1_000_000, **kw))
        r1[name] = {"ms": round(ms, 1), "cycles": infos[0].cycles, "sweeps": infos[0].sweeps,
                    "all_copies_same_cycles": all(i.cycles == infos[0].cycles for i in infos)}
        # each one-workgroup row against the per-step run of the same cycle shape
        if name in ("global", "overlap_t256_s32_o62"):
            x_steps = xs[0].clone()
        elif name.endswith("one_workgroup"):
            r1[name]["iterate_equals_per_step_run"] = bool(torch.equal(xs[0], x_steps))
        log(f"replica R1 {name}: {ms:.1f} ms, {infos[0].cycles} cycles")
    r1["speedup_paper_setting"] = round(r1["global"]["ms"] / r1["paper_t32_s16"]["ms"], 2)
    r1["speedup_paper_overlap_setting"] = round(r1["global"]["ms"] / r1["paper_t32_s16_o4"]["ms"], 2)
    r1["paper_reported"] = {"t32_s16": 3.79, "t32_s16_o4": 8.00, "note": "the paper's Tables 1 and 2, its own GPU"}
    r1["speedup_overlap"] = round(r1["global"]["ms"] / r1["overlap_t256_s32_o62"]["ms"], 2)
    assert r1["global_one_workgroup"]["cycles"] == r1["global"]["cycles"]
    r1["speedup_overlap_one_workgroup_vs_global_one_workgroup"] = round(
        r1["global_one_workgroup"]["ms"] / r1["overlap_t256_s32_o62_one_workgroup"]["ms"], 2)
    r1["hbm_pass_ratio_paper_setting"] = round(r1["global"]["cycles"] / r1["paper_t32_s16"]["cycles"], 2)
    r1["note"] = ("every batched step is a cycle launch plus a judge launch over all copies, so the s = 1 "
                  "steps of the global run pay the judge 128 760 times; the pass ratio is the paper's "
                  "measure of work.  The one-workgroup rows run each copy's whole solve inside one "
                  "workgroup (HJ_BATCH_WG1D): one launch, iterates in LDS; global_one_workgroup is "
                  "classical Jacobi that way (s = 1 cycles without overlap are classical sweeps), the "
                  "like-for-like baseline of the one-workgroup overlap row")
    out["r1_1d_1024_copies"] = r1

    F2 = torch.ones((n, n), dtype=torch.float64, device="cuda")
    X2 = torch.empty_like(F2)
    r2 = {"workload": "2D -lap u = 1 on 1024^2, x0 = 1, to 1e-4"}
    tile2, s2, ov2, _ = hj.autotune(2, n, n)
    # the right-hand-side tuner: trial solves of this problem to the same
    # tolerance, inexact overlaps included (its own time is reported apart)
    X2.fill_(1.0)
    tune_ms, (tile3, s3, ov3, trial_ms) = timed(lambda: hj.autotune_solve(F2, X2, h, trial_tol=1e-4))
    for name, kw in (("global", dict(method="global")),
                     ("paper_t32x32_s16", dict(tile=(32, 32), s=16, overlap=(0, 0))),
                     ("paper_t32x32_s32_o4", dict(tile=(32, 32), s=32, overlap=(4, 4))),
                     ("overlap_autotuned_exact_regime", dict(tile=tile2, s=s2, overlap=ov2)),
                     ("overlap_autotuned", dict(tile=tile3, s=s3, overlap=ov3))):
        X2.fill_(1.0)
        ms, info = timed(lambda: hj.solve_2d(F2, X2, h, rel_tol=1e-4, max_cycles=1_000_000, **kw))
        r2[name] = {"ms": round(ms, 1), "cycles": info.cycles, "sweeps": info.sweeps}
        if name == "overlap_autotuned_exact_regime":
            r2[name].update(tile=list(tile2), s=s2, overlap=list(ov2), by="hj_autotune (o = 2s - 2, time per sweep)")
        if name == "overlap_autotuned":
            r2[name].update(tile=list(tile3), s=s3, overlap=list(ov3), tuning_ms=round(tune_ms, 1),
                            by="hj_autotune_solve (trial solves of this problem to 1e-4, inexact overlaps included)")
        log(f"replica R2 {name}: {ms:.1f} ms, {info.cycles} cycles")
    r2["speedup_paper_setting"] = round(r2["global"]["ms"] / r2["paper_t32x32_s16"]["ms"], 2)
    r2["speedup_paper_overlap_setting"] = round(r2["global"]["ms"] / r2["paper_t32x32_s32_o4"]["ms"], 2)
    r2["paper_reported"] = {"t32x32_s16": 3.98, "t32x32_s32_o4": 5.84, "note": "the paper's Tables 3 and 4, its own GPU"}
    r2["speedup_overlap"] = round(r2["global"]["ms"] / r2["overlap_autotuned"]["ms"], 2)
    r2["speedup_overlap_exact_regime"] = round(r2["global"]["ms"] / r2["overlap_autotuned_exact_regime"]["ms"], 2)
    r2["hbm_pass_ratio_paper_setting"] = round(r2["global"]["cycles"] / r2["paper_t32x32_s16"]["cycles"], 2)
    out["r2_2d_1024"] = r2
    return out


def diffusion_rows(torch, hj, stream):
    """Variable-coefficient diffusion -div(a grad u) = f, a = exp(g) with g a
    squared-exponential Gaussian random field (length 0.05, variance 1).
    (1) Cycle throughput of the VC kernel at 1024^2 (fixed cycles, one RHS).
    (2) The autograd pipeline at 64^2 with 16 right-hand sides: forward solve
    to 1e-10, loss mean (u - t)^2 with t smooth, backward = adjoint solve to
    1e-10 and dL/da, dL/df.  (3) Central differences (eps 1e-6, FP64) of the
    loss on 32 entries of a and 8 of f at 32^2 with 2 right-hand sides.  The
    1024^2 solves to 1e-10 are out of reach for any Jacobi-type iteration when
    the adjoint right-hand side is smooth, hence the smaller grids for (2)/(3)."""
    from paper_2006_16465_amd import workloads as W
    out = {}
    shape = dict(tile=(64, 32), s=8, overlap=(14, 14))
    log("differentiable: VC cycle throughput at 1024^2")
    n = 1024
    h = 1.0 / (n + 1)
    a = torch.from_numpy(W.diffusion_coefficient(n, 0.05, 1.0, 7)).cuda()
    f = torch.from_numpy(W.rhs_2d_modes(n, n, 8, 0.0, 0)).cuda()[None]
    u = torch.zeros_like(f)
    K = 40

    def vc_cycle_us(lds):
        # best of 3 fixed-cycle solves (the events also carry the gaps
        # between launches)
        hj.solve_vc_2d(a, f, u, h, rel_tol=0.0, max_cycles=4, lds_kernel=lds, **shape)
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            u.zero_()
            e0.record(stream)
            hj.solve_vc_2d(a, f, u, h, rel_tol=0.0, max_cycles=K, lds_kernel=lds, **shape)
            e1.record(stream)
            e1.synchronize()
            t = e0.elapsed_time(e1) * 1e3 / K
            best = t if best is None else min(best, t)
        return best

    us, us_lds = vc_cycle_us(False), vc_cycle_us(True)
    vbytes = vc_cycle_bytes(n, n, shape["tile"], shape["overlap"])
    out["vc_cycle_1024"] = {"tile": list(shape["tile"]), "s": shape["s"], "overlap": list(shape["overlap"]),
                            "us_per_cycle": round(us, 1), "gsweeps_per_s": round(n * n * shape["s"] / us / 1e3, 1),
                            "body": "register-resident tiles",
                            "us_per_cycle_lds_body": round(us_lds, 1),
                            "algorithmic_bytes_per_cycle": vbytes,
                            "achieved_gbs": round(vbytes / us / 1e3, 1),
                            "frac_of_hbm_peak": round(vbytes / us / 1e3 / HBM_PEAK_GBS, 3)}

    # the configuration's own size, 16 right-hand sides: measured cycle rate
    # of the batched forward and adjoint solves and a projection of the time
    # to 1e-10 from the per-cycle residual factor between cycles c1 and c2
    log("differentiable: 1024^2 x 16 forward and adjoint, rate-based projection to 1e-10")
    B, c1, c2 = 16, 500, 1500
    F16 = torch.from_numpy(np.stack([W.rhs_2d_modes(n, n, 8, 0.0, b) for b in range(B)])).cuda()
    U16 = torch.zeros_like(F16)
    T16 = torch.from_numpy(np.stack([W.smooth_modes_2d(n, 3, 3, 100 + b) for b in range(B)]) * 1e-3).cuda()

    def capped(solve, cycles):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        infos = solve(cycles)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1), [i.rel_residual for i in infos]

    def project(solve, what):
        t1, r1 = capped(solve, c1)
        t2, r2 = capped(solve, c2)
        per_cycle_ms = (t2 - t1) / (c2 - c1)
        proj = []
        for a1, a2 in zip(r1, r2):
            if a2 <= 1e-10:
                proj.append(c2)
                continue
            rho = (a2 / a1) ** (1.0 / (c2 - c1))
            proj.append(float("inf") if rho >= 1.0 else c2 + np.log(1e-10 / a2) / np.log(rho))
        worst = max(proj)
        finite = np.isfinite(worst)
        log(f"differentiable: {what}: rel residuals at {c1}: {r1}; at {c2}: {r2}")
        return {"batch": B, "cycles_measured": [c1, c2], "ms_per_cycle_batch": round(per_cycle_ms, 3),
                "gsweeps_per_s": round(B * n * n * shape["s"] / per_cycle_ms / 1e6, 1),
                "achieved_gbs": round(B * vbytes / per_cycle_ms / 1e6, 1),
                "rel_residual_at_c1_max": max(r1), "rel_residual_at_c2_max": max(r2),
                "per_cycle_factor_worst": max((b2 / b1) ** (1.0 / (c2 - c1)) for b1, b2 in zip(r1, r2)),
                "projected_cycles_to_1e-10": round(worst) if finite else None,
                "projected_s_to_1e-10": round(worst * per_cycle_ms * 1e-3, 1) if finite else None,
                "what": what}

    def fwd(cycles):
        U16.zero_()
        return hj.solve_vc_2d(a, F16, U16, h, rel_tol=1e-10, max_cycles=cycles, allow_not_converged=True, **shape)

    out["config_1024x16_forward"] = project(fwd, "forward solve, 16 random-mode right-hand sides")
    DL16 = 2.0 * (U16 - T16) / U16.numel()
    L16 = torch.zeros_like(F16)

    def adj(cycles):
        L16.zero_()
        return hj.solve_adjoint(a, U16, DL16, L16, h, rel_tol=1e-10, max_cycles=cycles, grad_a=False,
                                allow_not_converged=True, **shape)[0]

    out["config_1024x16_adjoint"] = project(adj, "adjoint solve, dL/du = 2 (u - t) / N with t smooth")
    # a smooth right-hand side sits in the slowest modes: with a = 1 the
    # smoothest Jacobi mode decays by cos(pi h) per sweep, so a cycle of s
    # exact sweeps gains cos(pi h)^s; the variable coefficient only slows it
    lb = int(np.ceil(np.log(1e-10) / (shape["s"] * np.log(np.cos(np.pi * h)))))
    adj_row = out["config_1024x16_adjoint"]
    adj_row["cycles_to_1e-10_if_a_were_1"] = lb
    adj_row["s_to_1e-10_if_a_were_1"] = round(lb * adj_row["ms_per_cycle_batch"] * 1e-3, 1)
    log(f"differentiable: {out['config_1024x16_forward']}; {out['config_1024x16_adjoint']}")
    del F16, U16, T16, DL16, L16

    def pipeline(n, batch, tol, seed):
        h = 1.0 / (n + 1)
        a0 = torch.from_numpy(W.diffusion_coefficient(n, 0.05, 1.0, seed)).cuda()
        f0 = torch.from_numpy(np.stack([W.rhs_2d_modes(n, n, 8, 0.0, seed + b) for b in range(batch)])).cuda()
        t = torch.from_numpy(np.stack([W.smooth_modes_2d(n, 3, 3, seed + b) for b in range(batch)]) * 1e-3).cuda()
        return h, a0, f0, t

    log("differentiable: forward + adjoint at 64^2, 16 right-hand sides")
    h, a0, f0, t = pipeline(64, 16, 1e-10, 11)
    opts = dict(h=h, rel_tol=1e-10, **shape)
    A = a0.clone().requires_grad_(True)
    F = f0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U = hj.diffusion_solve(F, A, **opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = torch.mean((U - t) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["pipeline_64"] = {"batch": 16, "tol": 1e-10, "forward_ms": round((t1 - t0) * 1e3, 1),
                          "backward_ms": round((t2 - t1) * 1e3, 1),
                          "grad_a_norm": float(A.grad.norm()), "grad_f_norm": float(F.grad.norm())}

    log("differentiable: central differences at 32^2 on 32 entries of a and 8 of f")
    h, a0, f0, t = pipeline(32, 2, 1e-13, 21)
    opts = dict(h=h, rel_tol=1e-13, **{**shape, "tile": (32, 32), "overlap": (14, 14)})
    A = a0.clone().requires_grad_(True)
    F = f0.clone().requires_grad_(True)
    torch.mean((hj.diffusion_solve(F, A, **opts) - t) ** 2).backward()
    ga, gf = A.grad.cpu().numpy(), F.grad.cpu().numpy()
    rng = np.random.default_rng(0)
    eps = 1e-6
    err_a, err_f = 0.0, 0.0
    with torch.no_grad():
        def loss_of(aa, ff):
            return torch.mean((hj.diffusion_solve(ff, aa, **opts) - t) ** 2).item()
        for _ in range(32):
            r, q = rng.integers(0, 34), rng.integers(0, 34)
            ap, am = a0.clone(), a0.clone()
            ap[r, q] += eps
            am[r, q] -= eps
            fd = (loss_of(ap, f0) - loss_of(am, f0)) / (2 * eps)
            err_a = max(err_a, abs(fd - ga[r, q]))
        for _ in range(8):
            b, r, q = rng.integers(0, 2), rng.integers(0, 32), rng.integers(0, 32)
            fp, fm = f0.clone(), f0.clone()
            fp[b, r, q] += eps
            fm[b, r, q] -= eps
            fd = (loss_of(a0, fp) - loss_of(a0, fm)) / (2 * eps)
            err_f = max(err_f, abs(fd - gf[b, r, q]))
    out["finite_differences_32"] = {"entries_a": 32, "entries_f": 8, "eps": eps,
                                    "max_err_a_rel_to_max_grad": float(err_a / np.abs(ga).max()),
                                    "max_err_f_rel_to_max_grad": float(err_f / np.abs(gf).max())}
    log(f"differentiable: {out}")
    return out


def calibrate_copy(torch):
    """A plain copy of 2^27 doubles (1 GiB read + 1 GiB written) three times,
    to scale FETCH_SIZE / WRITE_SIZE counter readings to bytes."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                      "launches": 3}), flush=True)


def cpu_baseline(args, W, cycles_h, tile, ov, s, seed_ms_h):
    """The CPU oracle, as it stands (OpenMP over tiles, residual checked every
    cycle), on the benchmark's own workload: the hierarchical solve of every
    seed to the same tolerance with the same tile, s and overlap, timed whole
    (no scaling); classical Jacobi on the two seeds that need the fewest
    sweeps as context.  A reported baseline, not a target."""
    import oracle
    n = args.n
    h = W.grid_h(n)
    oracle._load()
    log("cpu baseline: full oracle solves ...")
    per_seed, cyc = {}, {}
    for sd in args.seeds:
        f = W.rhs_2d_modes(n, n, 8, 0.0, sd)
        t0 = time.perf_counter()
        _, c, _, _ = oracle.solve_2d(f, np.zeros_like(f), h, h, tile=tile, s=s, tol=args.tol, overlap=ov)
        per_seed[str(sd)] = round((time.perf_counter() - t0) * 1e3, 1)
        cyc[str(sd)] = c
    classical = {}
    for sd in (0, 1):
        f = W.rhs_2d_modes(n, n, 8, 0.0, sd)
        t0 = time.perf_counter()
        _, c, _, _ = oracle.solve_2d(f, np.zeros_like(f), h, h, method=oracle.CLASSICAL, tol=args.tol)
        classical[str(sd)] = {"ms": round((time.perf_counter() - t0) * 1e3, 1), "sweeps": c}
    mean_ms = float(np.mean(list(per_seed.values())))
    gpu_ms = float(np.mean(seed_ms_h))
    return {
        "value": round(mean_ms, 1), "unit": "ms", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": f"the whole workload: hierarchical solves of seeds {args.seeds} to {args.tol:g} "
                  f"(tile {list(tile)}, s {s}, overlap {list(ov)}), each timed once; "
                  f"mean ms per problem like value",
        "ms_per_seed": per_seed, "cycles_per_seed": cyc,
        "cycles_equal_gpu": [cyc[str(sd)] for sd in args.seeds] == list(cycles_h),
        "classical_seeds_0_1": classical,
        "gpu_speedup_over_oracle": round(mean_ms / gpu_ms, 1),
    }


if __name__ == "__main__":
    main()
