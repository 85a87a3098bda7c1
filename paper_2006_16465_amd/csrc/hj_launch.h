// hj_launch.h -- host-side launchers of the HIP kernels (internal to libhj).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hj_device.h"

namespace hj {

enum Dtype : int { F64 = 0, F32 = 1 };

// 2D problem geometry and coefficients (row-major, leading dimension ld).
struct Geom2 {
    int nx, ny;
    int64_t ld;
    int tx, ty, ox, oy;  // tile extents and overlaps
    int ntx, nty;        // tiles per axis
    int iso;             // hx == hy: use the h^2 f form of the update
    int reg;             // allow the register-resident cycle kernel (full tiles only)
    double hh;           // h^2 (iso)
    double wx, wy, dinv; // 1/hx^2, 1/hy^2, 1/(2wx + 2wy)
};

struct Geom1 {
    int64_t n;
    int t, o;
    int64_t nt;          // tiles
    double hh;           // h^2
    double w1;           // 1/h^2
};

bool cycle2d_supported(int tx, int ty);
// false when the tile shape has no kernel for this grid (a 128 extent needs
// the register kernel and a grid of at least one full tile)
bool cycle2d_runnable(const Geom2 &g);
bool cycle1d_supported(int t);

// Number of workgroups (= reduction partials) each launcher uses.
int64_t cycle2d_blocks(const Geom2 &g);
int64_t sweep2d_blocks(const Geom2 &g);
int64_t resid2d_blocks(const Geom2 &g);
int64_t cycle1d_blocks(const Geom1 &g);
int64_t sweep1d_blocks(const Geom1 &g);
int64_t resid1d_blocks(const Geom1 &g);

// One hierarchical cycle xin -> xout.  res: also reduce ||f - A xin||^2 into
// red.part_cur, judge iterate red.c - 1 from red.part_prev (workgroup 0), and
// skip all work once red.ctrl->status is set.
hipError_t launch_cycle2d(int dt, const Geom2 &g, int s, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st);
// One classical sweep over the whole grid, same residual contract.
hipError_t launch_sweep2d(int dt, const Geom2 &g, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st);
// Residual of x (optionally stored to r_out); partial sums of ||r||^2 into part.
hipError_t launch_resid2d(int dt, const Geom2 &g, const void *f, const void *x, void *r_out,
                          double *part, hipStream_t st);

hipError_t launch_cycle1d(int dt, const Geom1 &g, int s, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st);
hipError_t launch_sweep1d(int dt, const Geom1 &g, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st);
hipError_t launch_resid1d(int dt, const Geom1 &g, const void *f, const void *x, void *r_out,
                          double *part, hipStream_t st);

// Whole 1D hierarchical solve in one workgroup (register tiles of 64..512
// points, at most 16 tiles, f and two iterates in LDS).  Runs cycles
// [c_begin, c_end) (c_end <= maxc + 1) on x in place, carrying the solve state
// in ctrl from one launch to the next; every: judge every iterate (tolerance
// mode), else only iterates 0 and maxc.
bool solve1d_wg_supported(const Geom1 &g, int dt);
// One problem of a one-workgroup batch (its own grid, f and x).
struct WgProb {
    Geom1 g;
    const void *f;
    void *x;
};
// Workgroup b solves probs[b] (device array) with state ctrls[b]; every
// problem passes solve1d_wg_supported with tile tt; max_n, max_nt: the
// largest n and tile count over the batch.
hipError_t launch_solve1d_wg_batch(int dt, int tt, const WgProb *probs, int64_t nprob, int64_t max_n,
                                   int64_t max_nt, int s, int64_t c_begin, int64_t c_end, int64_t maxc, double tol,
                                   bool every, Ctrl *ctrls, hipStream_t st);
hipError_t launch_ctrl_init_n(Ctrl *ctrls, int64_t n, hipStream_t st);
hipError_t launch_solve1d_wg(int dt, const Geom1 &g, int s, const void *f, void *x, int64_t c_begin,
                             int64_t c_end, int64_t maxc, double tol, bool every, Ctrl *ctrl, hipStream_t st);

// Sum n partials and judge iterate c (one workgroup).
hipError_t launch_judge(const double *part, int n, Ctrl *ctrl, int64_t c, double tol, hipStream_t st);

// sw_tol >= 0: hand-over point of the solve (see Ctrl)
hipError_t launch_ctrl_init(Ctrl *ctrl, hipStream_t st, double sw_tol = -1.0, int64_t sw_min_c = 0);

// variable-coefficient diffusion (hj_vc.hip)
struct GeomVC {
    int nx, ny;
    int64_t ld;
    int tx, ty, ox, oy, ntx, nty;
    const double *a;  // (ny+2) x lda node coefficients
    int64_t lda;
    double ihx2, ihy2;
    int reg;          // 1: register-resident tiles where the grid holds a full tile
};
int64_t cycle_vc_blocks(const GeomVC &g);
int64_t sweep_vc_blocks(const GeomVC &g);
hipError_t launch_cycle_vc(const GeomVC &g, int s, bool res, const double *f, const double *xin,
                           double *xout, const Red &red, double tol, hipStream_t st);
hipError_t launch_sweep_vc(const GeomVC &g, bool res, const double *f, const double *xin, double *xout,
                           const Red &red, double tol, hipStream_t st);
hipError_t launch_resid_vc(const GeomVC &g, const double *f, const double *x, double *r_out,
                           double *part, hipStream_t st);
hipError_t launch_grad_a_vc(const GeomVC &g, const double *u, const double *lam, int nb,
                            int64_t bstride, double *grad, int64_t ldg, hipStream_t st);

// ---------------------------------------------------------------- batches
// One problem of a batch on the device.  Main buffers: 0 is the caller's x,
// 1 a scratch array of the same layout.  A refined problem also has an FP32
// residual r32 and two FP32 correction buffers e0 / e1, all with the pitch of
// x.  Work items: 2D tiles, 1D tile groups; a refinement step splits the grid
// into blocks (2D 64 columns x 32 rows, 1D 2048 points) dealt round-robin to
// the problem's work items.
struct BProb {
    int32_t dim;         // 1, 2, or 3 (2D variable coefficient, FP64, plain)
    int32_t dt;          // F64 / F32: precision of f and x (the main cycles)
    Geom2 g2;            // dim 2
    Geom1 g1;            // dim 1
    GeomVC gv;           // dim 3
    const void *f;
    void *x;
    void *s1;
    float *r32, *e0, *e1;  // refined problems only
    int64_t item0;       // first work item of this problem in its list
    int64_t nitems;      // work items
    int64_t part0;       // first partial slot (one per work item)
    int64_t rnitems;     // refinement-step blocks
    double tol;          // relative tolerance (<= 0: run max_cycles cycles)
    int64_t max_cycles;  // cycles a result may take (all phases together)
    int32_t s;           // sweeps per cycle
    int32_t pad;
};

// Phases of a problem.  MAIN: cycles of the problem's own precision on x.
// INNER: FP32 cycles on the correction equation A e = r32.  REF: one step of
// refinement (x += e, the FP64 residual of the new x, r32 and a cleared
// correction for the next INNER phase) in place of a cycle; `next` says what
// follows it (END: nothing, the budget is spent).
enum : int32_t { PH_MAIN = 0, PH_INNER = 1, PH_REF = 2, PH_END = 3 };

// Per-problem state, written by the judge (and init) only.
struct BState {
    double r0sq;      // ||f - A x_0||^2
    double rsq;       // ||f - A x||^2 of the latest FP64-judged x
    double in_tolsq;  // INNER: stop once ||r32 - A e_j||^2 <= in_tolsq
    double mark_rsq;  // MAIN: residual where the rate measurement starts; INNER: last halving
    double lnrate;    // ln of the per-cycle residual factor at the switch (0: unknown)
    int64_t j;        // iterate of the current phase that the next cycle reads
    int64_t mark_j;   // cycle of mark_rsq (-1: none)
    int64_t used;     // cycles inside the result (closed phases)
    int32_t status;   // ST_*
    int32_t phase;    // PH_*
    int32_t xsel;     // main buffer holding iterate 0 of the main phase, or the refined x
    int32_t esel;     // inner buffer holding iterate 0 of the inner phase
    int32_t rx;       // REF: main buffer with x (the new x goes to xsel)
    int32_t esrc;     // REF: inner buffer with e (-1: none)
    int32_t next;     // REF: phase after the step
    int32_t outer;    // correction solves taken
    int32_t cont;     // main phase runs to rel_tol (no switch to FP32)
    int32_t pad;
};

// Refinement settings of a batch (refine = 0: plain solves).
struct BRefine {
    int32_t refine;
    int32_t max_outer;  // correction solves per problem; then it continues in FP64
    double switch_tol;  // MAIN -> refinement at most at this relative residual
    double inner_min;   // least relative reduction one correction solve is asked for
    double fmax;        // predicted FP32 floor above which a problem stays FP64
};

struct BatchLaunch {
    const BProb *probs;
    const int32_t *owner;  // problem of each work item
    int64_t nitems;
    const BState *state;   // one per problem
    double *part;          // one partial slot per work item
    int s;
};

int64_t ref_items(int dim, int64_t nx, int64_t ny);
bool batch2d_supported(int tx, int ty);
// iso: the work list holds only problems with hx == hy (else only the others).
// Plain batches run cycles of precision dt; refined ones (FP64 problems) run
// each problem's phase: FP64 main cycle, FP32 inner cycle or refinement step.
hipError_t launch_batch_cycle2d(int dt, bool refine, int tx, int ty, bool iso, const BatchLaunch &L,
                                hipStream_t st);
hipError_t launch_batch_cycle1d(int dt, bool refine, int t, const BatchLaunch &L, hipStream_t st);
bool batch_vc_supported(int tx, int ty);
hipError_t launch_batch_cycle_vc(int tx, int ty, const BatchLaunch &L, hipStream_t st);
hipError_t launch_batch_judge(const BProb *probs, int nprob, BState *state, const double *part,
                              const BRefine &rf, hipStream_t st);
hipError_t launch_batch_init(BState *state, int nprob, hipStream_t st);
// copies each stopped problem's result into x when it sits in buffer 1
hipError_t launch_batch_finalize(const BProb *probs, int nprob, const BState *state, hipStream_t st);

// mixed precision helpers (hj_refine.hip)
int64_t resid2d_mixed_blocks(const Geom2 &g);
hipError_t launch_resid2d_f64_to_f32(const Geom2 &g, const double *f, const double *x, float *r32,
                                     float *e32, double *part, hipStream_t st);
hipError_t launch_axpy_f32_to_f64(const Geom2 &g, const float *e, double *x, hipStream_t st);

}  // namespace hj
