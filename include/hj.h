/*
 * hj.h -- C ABI of the MI355X (gfx950) hierarchical Jacobi library (libhj.so).
 *
 * Method: Islam & Wang, "Hierarchical Jacobi Iteration for Structured Matrices
 * on GPUs using Shared Memory" (arXiv:2006.16465).
 *
 * Problems solved (Sec. 3.4 and Sec. 4.2): the finite-difference Poisson
 * systems A x = f with homogeneous Dirichlet boundaries,
 *   1D:  -u'' = f on [0,1], A = tridiag(-1, 2, -1) / h^2, n interior points;
 *   2D:  -(u_xx + u_yy) = f on [0,1]^2, 5-point stencil with weights
 *        1/hx^2 (x neighbours) and 1/hy^2 (y neighbours), diagonal
 *        2/hx^2 + 2/hy^2, nx * ny interior points.
 *
 * Iterations:
 *   HJ_GLOBAL       classical Jacobi (Sec. 2.1 elemental update, Sec. 3.2 / 4.2
 *                   global-memory GPU version): one sweep of the whole grid per
 *                   cycle.
 *   HJ_HIERARCHICAL the hierarchical cycle (Sec. 3.3 three steps; Sec. 4.1 in
 *                   2D): each tile plus a one-point halo is copied on chip, s
 *                   Jacobi sub-iterations run on the tile interior with the halo
 *                   frozen at the previous global iterate, and the interior is
 *                   written to a second global array.  With overlap o > 0
 *                   (Sec. 3.5 / 4.3) neighbouring tiles share o interior points
 *                   and each shared point is written by the tile in which it is
 *                   farther from the frozen edge.  s = 1 reproduces classical
 *                   Jacobi iterates exactly.
 *
 * Tile partition of an axis of n points (tile t, overlap o, 0 <= o < t): if
 * n <= t, one tile covers all points; otherwise ceil((n - o) / (t - o)) full
 * tiles at stride t - o, the last moved left so that it ends at point n.  Where
 * two neighbours overlap in [a, b) the left tile writes the first
 * ceil((b - a) / 2) points.  The 2D partition is the product of the per-axis
 * partitions.
 *
 * Arithmetic (IEEE round-to-nearest, no flush to zero; the compiler does not
 * contract to fused multiply-add):
 *   1D:          x_i <- (h^2 f_i + (x_{i-1} + x_{i+1})) * 0.5
 *   2D, hx==hy:  x   <- (h^2 f + ((x_W + x_E) + (x_S + x_N))) * 0.25
 *   2D, hx!=hy:  x   <- (f + (wx (x_W + x_E) + wy (x_S + x_N))) * dinv
 * with h^2 f rounded once, wx = 1/hx^2, wy = 1/hy^2, dinv = 1/(2 wx + 2 wy),
 * W/E the x neighbours (same row), S/N the y neighbours (adjacent rows).  The
 * register-resident kernels evaluate the first two as one fused multiply-add
 * of the neighbour sum with the exact factor 0.5 / 0.25 and the prescaled
 * h^2 f * 0.5 / * 0.25; scaling by a power of two commutes with rounding, so
 * this is the two-step result bit for bit whenever the values involved are
 * normal numbers (magnitudes above 2^-1020 in FP64, 2^-124 in FP32; subnormal
 * intermediates can differ in the last place).  In FP64 the iterates are
 * therefore bit-reproducible and independent of the order in which tiles run.
 *
 * Residual: r = f - A x over the interior, its 2-norm accumulated in FP64 with
 * a fixed-order reduction (deterministic run to run).  A solve stops at the
 * first cycle c with ||r_c||_2 <= rel_tol * ||r_0||_2 (the paper's stopping
 * rule, Sec. 3.4, with the factor 1e-4 replaced by rel_tol); the residual is
 * evaluated for every cycle on the global iterate, fused into the next
 * cycle's tile load.
 *
 * Memory layout: all arrays are device memory of the selected dtype.  1D
 * arrays hold the n interior points contiguously.  2D arrays are row-major
 * with leading dimension ld >= nx elements: point (row y = j, column x = i) is
 * at [j * ld + i]; f, x and r_out share ld.  Columns nx..ld-1 are never read
 * or written.  Pointers must be aligned to the element size.
 *
 * Ownership: the caller owns f, x and r_out.  The library owns its scratch
 * (one second iterate array of the same size as x, and a few KB of reduction
 * partials and control words), allocated on first use per device and size and
 * kept until the process ends.  Calls are synchronous with respect to the
 * stream passed in: they enqueue work on it and return after it has drained.
 * Calls from several host threads on one device are serialised internally.
 *
 * Errors: every entry point validates its arguments before any HIP call and
 * returns a status; no C++ exception crosses the ABI.  hj_last_error() gives a
 * detail string for the last failing call of the calling thread.
 */
#ifndef HJ_H
#define HJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The *_RANGE_MIN / *_RANGE_MAX names of the enums below are not values to
 * pass: they widen each type to the whole int32 range, so that any integer a
 * caller passes is a valid value of the type (an invalid one is rejected with
 * HJ_ERR_INVALID_ARG, or named "unknown status"). */
typedef enum hj_status {
    HJ_OK = 0,
    HJ_ERR_INVALID_ARG = 1,   /* argument validation failed; nothing was run */
    HJ_ERR_NOT_CONVERGED = 2, /* max_cycles reached; x and info hold the last iterate */
    HJ_ERR_NONFINITE = 3,     /* a residual norm became NaN/Inf; x holds that iterate */
    HJ_ERR_UNSUPPORTED = 4,   /* valid but not provided (tile shape, entry point) */
    HJ_ERR_HIP = 5,           /* a HIP runtime call failed; see hj_last_error() */
    HJ_STATUS_RANGE_MIN = -2147483647 - 1,
    HJ_STATUS_RANGE_MAX = 2147483647
} hj_status;

typedef enum hj_dtype {
    HJ_F64 = 0,
    HJ_F32 = 1,
    HJ_DTYPE_RANGE_MIN = -2147483647 - 1,
    HJ_DTYPE_RANGE_MAX = 2147483647
} hj_dtype;

typedef enum hj_method { HJ_HIERARCHICAL = 0, HJ_GLOBAL = 1 } hj_method;

/* hj_params.flags: run every 2D cycle (constant- and variable-coefficient)
 * on the LDS ping-pong kernel instead of the register-resident one (same
 * iterates; for comparison and testing). */
#define HJ_FLAG_LDS_KERNEL 0x1
/* hj_params.flags, 1D solves: one kernel launch per cycle (HJ_GLOBAL: per
 * sweep) even where one workgroup can run the whole solve (same iterates; for
 * comparison and testing).  Without it, a 1D hierarchical solve with tiles of
 * 64, 128, 256 or 512 points, at most 16 tiles and 3 n element sizes within
 * the workgroup's LDS (150 KiB on gfx950: the device's opt-in limit per
 * workgroup less 1 KiB, at most 150 KiB; 60 KiB where the device reports no
 * opt-in limit) runs all its cycles inside one workgroup (Sec. 3.3 cycle,
 * global iterates in LDS, the residual judged on the device every cycle).
 * HJ_GLOBAL solves of such grids run the same way as cycles of one
 * sub-iteration without overlap on the smallest tile of 64..512 points that
 * covers the grid in at most 16 tiles: these are classical sweeps exactly
 * (Sec. 3.3, k = 1), so both methods pay the same (no) launch cost. */
#define HJ_FLAG_LAUNCH_PER_CYCLE 0x2

typedef struct hj_params {
    int32_t tile_x;      /* interior tile extent along x (1D: the tile); 0 = 32.
                            2D supports 16, 32, 64, 128 (x 16, 32, 64, 128; tile_x = 16
                            only with tile_y <= 64; a 128 extent needs a grid of at
                            least one full tile); 1D supports 32..1024 (powers of 2) */
    int32_t tile_y;      /* interior tile extent along y (2D); 0 = 32 */
    int32_t overlap_x;   /* interior points shared by x-neighbour tiles, 0 <= o < tile */
    int32_t overlap_y;   /* same along y */
    int32_t s;           /* sub-iterations per cycle (the paper's k), >= 1; ignored by HJ_GLOBAL */
    int32_t method;      /* hj_method */
    int64_t max_cycles;  /* >= 1: cycles (HJ_GLOBAL: sweeps) allowed */
    int32_t check_every; /* cycles enqueued between host polls of the device-side
                            convergence flag; 0 = adaptive (about 0.5 ms of GPU work
                            per poll).  Does not change results. */
    int32_t flags;       /* 0, or HJ_FLAG_LDS_KERNEL | HJ_FLAG_LAUNCH_PER_CYCLE */
    double rel_tol;      /* > 0: stop at the first cycle c with ||r_c|| <= rel_tol ||r_0||.
                            <= 0: run exactly max_cycles cycles with no residual
                            evaluation in between (fixed-count mode). */
} hj_params;

typedef struct hj_info {
    int64_t cycles;      /* index c of the iterate returned in x */
    int64_t sweeps;      /* Jacobi sweeps applied per point: cycles * s (HIERARCHICAL) or cycles */
    double rel_residual; /* ||f - A x_c|| / ||f - A x_0|| (0 if ||f - A x_0|| == 0) */
    double r0_norm;      /* ||f - A x_0||_2 */
} hj_info;

/* Fill *p with defaults: 32 (x 32) tiles, no overlap, s = 16, hierarchical,
 * max_cycles = 1000000, check_every = 0 (adaptive), rel_tol = 1e-6. */
void hj_params_default(hj_params *p);

/* 1D solve (Sec. 3).  n >= 1 interior points, spacing h > 0.  f: n values,
 * x: n values, in/out (x_0 in, x_cycles out).  stream: hipStream_t or NULL for
 * the null stream.  info may be NULL.  Returns HJ_OK on convergence (or after
 * max_cycles in fixed-count mode). */
hj_status hj_solve_1d(int64_t n, double h, hj_dtype dtype, const void *f, void *x,
                      const hj_params *p, void *stream, hj_info *info);

/* 2D solve (Sec. 4).  nx, ny >= 1, ld >= nx, hx, hy > 0; f and x: ny rows of
 * ld elements; x in/out. */
hj_status hj_solve_2d(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                      const void *f, void *x, const hj_params *p, void *stream, hj_info *info);

/* Allocation-free 2D solve, for callers that cannot allocate device or
 * pinned memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, validation, iterates, stopping rule,
 * info and statuses as hj_solve_2d, bit for bit.  It calls no hipMalloc,
 * hipHostMalloc, hipFree or event creation: its scratch (the control block,
 * the reduction partials and the two spare iterate arrays, 2 ny ld element
 * sizes plus a few KB) lives in one static device array of
 * HJ_NOALLOC_SCRATCH_BYTES in the library, which every device the library
 * runs on holds until the process ends.  A grid whose scratch exceeds that
 * size returns HJ_ERR_INVALID_ARG before any HIP call (FP64 grids up to
 * 2048 x 2048 fit; hj_last_error() states the bytes needed).  In tolerance
 * mode the host reads the control block after every batch of cycles with a
 * plain copy and a stream synchronisation (no lookahead).  All calls on one
 * device share that device's array: calls from several host threads are
 * serialised, but calls made on one device by other means at the same time
 * (another process's library instance does not share it) would race on it. */
#define HJ_NOALLOC_SCRATCH_BYTES (96ull << 20)
hj_status hj_solve_2d_noalloc(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                              const void *f, void *x, const hj_params *p, void *stream, hj_info *info);

/* Mixed precision 2D solve: FP32 hierarchical cycles inside FP64 iterative
 * refinement.  f, x: FP64 (x in/out, ld as in hj_solve_2d).
 *
 * Phase 1 runs FP64 cycles (inner's tile, overlap, s, method) on x until the
 * relative residual is <= switch_tol and keeps the iterate one cycle past
 * that one (already computed while the verdict was reached).
 * Phase 2 repeats refinement steps: form
 * r = f - A x in FP64 (stored as FP32), solve A e = r from e = 0 with FP32
 * cycles, accumulate x += e in FP64.  A step's FP32 solve stops when its
 * residual is <= max(inner.rel_tol * ||r||, rel_tol * ||r_0|| / 2), likewise
 * handing over one cycle more: the second term stops it once the outer
 * tolerance is met (with a factor 2 to spare), the first bounds what one step
 * asks of FP32 (1e-6 is a good choice); inner.max_cycles caps it.
 * The solve stops when the FP64 residual meets rel_tol.
 *
 * The cycle is a consistent stationary iteration, so restarting it on the
 * correction equation continues the same iteration.  FP32 rounding, however,
 * leaves error in the slowest modes of Jacobi's iteration matrix (the
 * smoothest and the most oscillatory), about 1e-6 times the residual at
 * which the FP32 phase starts; those modes then take as long to remove as
 * the slowest mode of the grid.  switch_tol keeps that residue below
 * rel_tol.  switch_tol = 0 selects min(1, 1e4 * rel_tol), or min(1, 1e5 *
 * rel_tol) in the exact regime (hierarchical, overlap >= 2s - 2 on both
 * axes, where a cycle is s classical sweeps); switch_tol >= 1 runs FP32 from
 * the start.
 *
 * Phase 1 runs toward rel_tol itself and hands over at the switch point only
 * if it took at least switch_min_cycles FP64 cycles to get there (0 = 8):
 * about as many remain from there to rel_tol, and for fewer the
 * refinement's extra passes cost more than its FP32 cycles save.  A solve
 * that does not hand over is hj_solve_2d's FP64 solve to rel_tol, iterate
 * for iterate, with outer = 0. */
typedef struct hj_refine_params {
    hj_params inner;     /* cycle shape for both phases; FP32 solve tolerances (inner.rel_tol > 0) */
    double rel_tol;      /* > 0: outer tolerance on ||f - A x||_2 / ||f - A x_0||_2 */
    double switch_tol;   /* >= 0: FP64 phase target (0 = default, see above) */
    int32_t max_outer;   /* >= 1: refinement steps */
    int32_t flags;       /* must be 0 */
    int32_t switch_min_cycles; /* >= 0: least FP64 cycles to the switch point for a hand-over (0 = 8) */
    int32_t pad;         /* ignored */
} hj_refine_params;

typedef struct hj_refine_info {
    int64_t outer;         /* refinement steps taken */
    int64_t inner_cycles;  /* FP32 cycles over all steps (iterates handed over, as above) */
    int64_t fp64_cycles;   /* FP64 cycles of phase 1 (index of the iterate handed over, or of
                              the result when there was no hand-over) */
    double rel_residual;   /* final FP64 relative residual */
    double r0_norm;        /* ||f - A x_0||_2 */
} hj_refine_info;

hj_status hj_solve_2d_refined(int64_t nx, int64_t ny, int64_t ld, double hx, double hy,
                              const double *f, double *x, const hj_refine_params *p,
                              void *stream, hj_refine_info *info);

/* Residual r = f - A x (Sec. 3.4 / 4.2 operator) and ||r||_2 (FP64).
 * dim = 1 (uses nx = n, ny and ld ignored, hx = h) or 2.  r_out (same dtype and
 * layout as x) may be NULL; norm2_out (host) may be NULL. */
hj_status hj_residual(int32_t dim, int64_t nx, int64_t ny, int64_t ld, double hx, double hy,
                      hj_dtype dtype, const void *f, const void *x, void *r_out,
                      double *norm2_out, void *stream);

/* ---------------------------------------------------------------- batches
 * Many independent problems, 2D and 1D, of uneven sizes, solved together:
 * every cycle is one launch over the tiles of all 2D problems (two when some
 * have hx != hy), one over the tile groups of all 1D problems, and one that
 * judges every problem; a fixed run of such cycles is captured once in a HIP
 * graph and replayed until every problem has stopped.  Each problem's iterates
 * equal those of its own hj_solve_2d / hj_solve_1d call with the same cycle
 * shape, bit for bit, and it stops at its own first cycle that meets rel_tol. */
typedef struct hj_problem {
    int32_t dim;        /* 1 or 2 */
    int32_t flags;      /* must be 0 */
    int64_t nx, ny, ld; /* 2D: ny rows of ld >= nx elements; 1D: n = nx (ny, ld ignored) */
    double hx, hy;      /* grid spacings (1D: hx), finite and > 0 */
    const void *f;      /* device pointer, the batch's dtype */
    void *x;            /* device pointer, in/out: x_0 in, the stopping iterate out */
} hj_problem;

#define HJ_BATCH_AUTOTUNE 0x1
#define HJ_BATCH_REFINE 0x2
/* 1D problems only, each solved inside one workgroup: one launch covers
 * every problem's cycles (in launches of up to 4096 cycles), the iterates and
 * f in LDS, as hj_solve_1d runs a small grid.  Needs p1 hierarchical with
 * tile_x in {64, 128, 256, 512} and every problem at most 16 tiles with 3 n
 * element sizes within the workgroup's LDS (as for HJ_FLAG_LAUNCH_PER_CYCLE
 * above); not with HJ_BATCH_AUTOTUNE or
 * HJ_BATCH_REFINE (HJ_ERR_UNSUPPORTED otherwise).  Iterates, cycle counts
 * and infos are those of each problem's own hj_solve_1d call.  graph_cycles
 * is ignored; the scratch is a device copy of the problem table and one
 * solve state per problem (no iterate arrays). */
#define HJ_BATCH_WG1D 0x4

typedef struct hj_batch_params {
    hj_params p2;         /* 2D cycle: tile_x in {32, 64}, tile_y in {16, 32, 64, 128},
                             overlap, s (register-resident tiles: every 2D problem needs
                             nx >= tile_x and ny >= tile_y); method HJ_HIERARCHICAL */
    hj_params p1;         /* 1D cycle: tile_x in 32..1024, overlap_x, s */
    double rel_tol;       /* per problem; <= 0: every problem runs exactly max_cycles cycles */
    int64_t max_cycles;   /* >= 1: cycles per problem (HJ_BATCH_REFINE: FP64 and FP32 cycles
                             of all phases together) */
    int32_t dtype;        /* hj_dtype of every f and x */
    int32_t graph_cycles; /* cycles per graph replay, 0 = 8, at most 1024 */
    int32_t flags;        /* HJ_BATCH_WG1D: see above.
                             HJ_BATCH_AUTOTUNE: choose p2 and p1 with hj_autotune (2D on the
                             largest 2D problem, tiles limited to the smallest);
                             HJ_BATCH_REFINE: FP64 problems (dtype HJ_F64, rel_tol > 0), each on
                             its own schedule: FP64 cycles down to min(1e4 rel_tol,
                             rel_tol / 8F) (F the problem's FP32 floor predicted from its
                             measured convergence rate), then refinement steps (x += e and
                             the FP64 residual in one pass) around FP32 correction cycles;
                             a problem whose F exceeds 1/80, or whose correction solve stops
                             converging, continues with FP64 cycles */
    int32_t max_outer;    /* HJ_BATCH_REFINE: FP32 correction solves per problem (0 = 8);
                             after them a problem continues with FP64 cycles */
} hj_batch_params;

/* Scratch: one iterate array per problem (the sum of the problems' sizes;
 * refined batches add an FP32 residual and two FP32 correction arrays per
 * problem), partials and per-problem states, kept per device and grown on
 * demand.  infos[i].cycles counts the cycles inside problem i's result (FP64
 * and FP32 together when refined).  infos
 * (nprob entries) may be NULL; problem i met rel_tol iff
 * infos[i].rel_residual <= rel_tol (NaN: its residual became non-finite).
 * Problems must not share x arrays.  Returns HJ_OK when every problem met rel_tol
 * (or ran max_cycles in fixed-count mode), HJ_ERR_NOT_CONVERGED if some
 * stopped at max_cycles (their latest iterate is in x), HJ_ERR_NONFINITE if
 * some residual became non-finite. */
hj_status hj_solve_batched(const hj_problem *probs, int64_t nprob, const hj_batch_params *p,
                           void *stream, hj_info *infos);

/* Autotuner.  With overlap o = 2s - 2 a cycle is exactly s classical sweeps
 * (no stale halo value reaches an owned point), so every such shape converges
 * at the same rate per sweep and the fastest is the one with the least time
 * per cycle divided by s.  Times a few cycles of each candidate -- 2D tiles
 * 32x32, 64x32, 32x64, 64x64, 32x128, 64x128 no larger than (nx, ny); 1D tiles
 * 64..1024 no larger than nx; s from 4 to 16 (2D) or 32 (1D) with 2s - 2 at
 * most the tile minus 2 -- on a scratch problem of the given size and dtype,
 * and returns the best shape in *best (hierarchical, other fields defaulted)
 * and its time per sweep in microseconds.  Results are cached per size. */
hj_status hj_autotune(int32_t dim, int64_t nx, int64_t ny, hj_dtype dtype, void *stream,
                      hj_params *best, double *us_per_sweep);

/* Shape tuning on the caller's own problem.  The exact-regime tuner above
 * ranks shapes by time per classical sweep; an overlap below 2s - 2 lets
 * stale halo values reach owned points, which on smooth error still gains
 * close to s classical sweeps per cycle at a fraction of the redundant work
 * (Sec. 3.5 Table 2, Sec. 4.3 Table 4), and on other right-hand sides stalls.
 * This tuner therefore solves the given 2D problem (f, starting from x0,
 * which is not modified) to trial_tol with each candidate shape and keeps
 * the one that got there first, by wall time on the stream:
 *   tiles 32x32, 64x32, 32x64, 64x64, 64x128 that fit the grid (or only
 *   (tile_x, tile_y) when given), s in {4, 8, 12, 16, 24, 32}, even overlaps
 *   below the tile: 2s - 2 (exact regime, tried first), then the near-exact
 *   2s - 6, 2s - 10, 3s/2 (rounded up to even), s + 6, s + 2, then 8, 4, 2,
 *   0.  Near-exact overlaps keep every owned point a few points inside the
 *   stale halo's reach, so the halo's influence on it after s sweeps is
 *   small; on many right-hand sides they need the exact regime's cycle
 *   count with less redundant loading, on some they stall: the trial on the
 *   caller's problem decides.
 * With nrhs > 1 every candidate solves each right-hand side in turn (all
 * from x0) and is scored by the sum of the times; a candidate that misses
 * trial_tol on any of them is dropped, so a shape that only suits some of
 * the caller's right-hand sides loses.
 * A candidate is skipped without a trial when its measured time per cycle
 * times the sum over right-hand sides of ceil(N / s) already exceeds the
 * best time, N being the classical sweep count the exact-regime trials
 * revealed for that right-hand side (a cycle gains at most s classical
 * sweeps); each trial is capped at the cycles that could still beat the
 * best, and at max_trial_cycles.  best gets the winner (hierarchical,
 * rel_tol = trial_tol, other fields defaulted), *best_ms its time (summed
 * over right-hand sides; may be NULL).  HJ_ERR_NOT_CONVERGED if no
 * candidate reached trial_tol within max_trial_cycles on every right-hand
 * side. */
typedef struct hj_tune_params {
    double trial_tol;         /* > 0: relative residual each trial solve must reach */
    int64_t max_trial_cycles; /* >= 1: cap per trial */
    int32_t tile_x, tile_y;   /* 0, 0: all candidate tiles; else only this tile (a 2D tile shape) */
    int32_t flags;            /* must be 0 */
    int32_t nrhs;             /* 0 or 1: f is one right-hand side; 2..1024: f holds nrhs of them */
    int64_t rhs_stride;       /* elements from one right-hand side to the next (>= ny * ld if nrhs > 1) */
} hj_tune_params;

hj_status hj_autotune_solve(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                            const void *f, const void *x0, const hj_tune_params *tp, void *stream,
                            hj_params *best, double *best_ms);

/* The cycle shapes hj_solve_batched with HJ_BATCH_AUTOTUNE uses for this
 * table: hj_autotune on the largest 2D problem with tiles no larger than the
 * smallest 2D problem (and tile_x <= 64), and on the largest 1D problem.
 * p2 / p1 may be NULL; a dimension the table lacks leaves its output as
 * hj_params_default fills it. */
hj_status hj_autotune_batch(const hj_problem *probs, int64_t nprob, hj_dtype dtype, void *stream,
                            hj_params *p2, hj_params *p1);

/* Variable-coefficient diffusion -div(a grad u) = f on the 2D grid (the
 * general pentadiagonal Jacobi of Sec. 4 with per-point coefficients), for a
 * batch of right-hand sides sharing a.  a holds node values on the
 * (ny+2) x (nx+2) grid including the boundary nodes; each face weight is the
 * arithmetic mean of its two nodes over h^2, so A is symmetric positive
 * definite for a > 0:
 *   (A u)_p = sum over the 4 faces of p: a_face (u_p - u_neighbour) / h^2,
 * u = 0 on the boundary.  Jacobi update u_p <- (f_p + sum a_face u_nb / h^2) /
 * sum a_face / h^2; the hierarchical cycle, overlap and stopping rule are
 * those of hj_solve_2d.  Tiles (tile_x, tile_y) from {16, 32, 64}^2; grids
 * holding a full tile in each direction run register-resident tiles (two
 * rows of tile_x / 16 points a lane), smaller ones, or any with
 * HJ_FLAG_LDS_KERNEL, the LDS ping-pong tile: same iterates either way. */
typedef struct hj_vc_problem {
    int64_t nx, ny;        /* interior grid */
    int64_t ld;            /* leading dimension of f, u, lam (elements, >= nx) */
    int64_t lda;           /* leading dimension of a (elements, >= nx + 2) */
    double hx, hy;
    const double *a;       /* (ny + 2) rows x lda: node coefficients, FP64, device */
    int32_t batch;         /* right-hand sides, >= 1 */
    int32_t flags;         /* must be 0 */
    int64_t batch_stride;  /* elements between consecutive right-hand sides, >= ny * ld */
} hj_vc_problem;

/* Solve A(a) u_b = f_b for every b (FP64; u in/out, one info per b when infos
 * is not NULL).  Returns the worst status over the batch. */
hj_status hj_solve_vc_2d(const hj_vc_problem *prob, const double *f, double *u, const hj_params *p,
                         void *stream, hj_info *infos);

/* dL/da for a loss L(u) with A(a) u = f, given the forward states u and the
 * adjoint states lam (A lam = dL/du), summed over the batch:
 *   dL/da_P = -1/2 sum over faces (P, Q) of (u_P - u_Q)(lam_P - lam_Q) / h^2
 * (u = lam = 0 on boundary nodes).  grad: (ny + 2) rows x ld_grad (>= nx + 2). */
hj_status hj_vc_grad_a(const hj_vc_problem *prob, const double *u, const double *lam, double *grad,
                       int64_t ld_grad, void *stream);

/* Backward pass of the variable-coefficient solve (A symmetric, so the adjoint
 * solve is a forward solve on dL/du): lam_b <- A^-1 dL/du_b (lam holds the
 * initial guess on entry), dL/df = lam, and dL/da into dl_da when not NULL. */
typedef struct hj_adjoint_desc {
    hj_vc_problem prob;
    const double *u;       /* converged forward states (batch) */
    const double *dl_du;   /* dL/du (batch) */
    double *lam;           /* in: initial guess; out: adjoint states = dL/df (batch) */
    double *dl_da;         /* out, may be NULL */
    int64_t ld_grad;       /* leading dimension of dl_da */
    hj_params params;      /* solver for A lam = dL/du */
} hj_adjoint_desc;

hj_status hj_solve_adjoint(const hj_adjoint_desc *d, void *stream, hj_info *infos);

/* Number of tiles (workgroups of the cycle kernel) along one axis; the same
 * partition rule the kernels use.  Returns -1 on invalid arguments. */
int64_t hj_axis_tiles(int64_t n, int32_t tile, int32_t overlap);

const char *hj_status_string(hj_status s);
const char *hj_last_error(void);   /* thread-local; "" if none */
const char *hj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HJ_H */
