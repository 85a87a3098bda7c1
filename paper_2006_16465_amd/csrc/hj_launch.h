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

// Sum n partials and judge iterate c (one workgroup).
hipError_t launch_judge(const double *part, int n, Ctrl *ctrl, int64_t c, double tol, hipStream_t st);

hipError_t launch_ctrl_init(Ctrl *ctrl, hipStream_t st);

// variable-coefficient diffusion (hj_vc.hip)
struct GeomVC {
    int nx, ny;
    int64_t ld;
    int tx, ty, ox, oy, ntx, nty;
    const double *a;  // (ny+2) x lda node coefficients
    int64_t lda;
    double ihx2, ihy2;
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

// mixed precision helpers (hj_refine.hip)
// ---------------------------------------------------------------- batches
// One problem of a batch on the device.  Buffer 0 is the caller's x, buffer 1
// a scratch array of the same layout; iterate c lives in buffer c & 1.
struct BProb {
    int32_t dim;     // 1 or 2
    int32_t pad;
    Geom2 g2;        // dim 2
    Geom1 g1;        // dim 1
    const void *f;
    void *x;
    void *s1;
    int64_t item0;   // first work item of this problem in its dimension's list
    int64_t nitems;  // work items: 2D tiles, or 1D tile groups
    int64_t part0;   // first residual partial slot
    double tol;      // relative tolerance (<= 0: run max_cycles cycles)
    int64_t max_cycles;  // this problem stops running after iterate max_cycles
};

struct BCtl {
    int64_t cycle;       // cycle the next kernels run (advanced on the device)
    int64_t max_cycles;  // largest per-problem cap (replays run to it)
};

struct BatchLaunch {
    const BProb *probs;
    const int32_t *owner;  // problem of each work item
    int64_t nitems;
    const BCtl *bc;
    const Ctrl *ctrl;      // one per problem
    double *part;          // 2 x npart partial slots (by cycle parity)
    int64_t npart;
    int s;
};

// One problem of a batched refinement step: FP64 f, x (pitch ld), FP32
// residual and correction (pitch nx).  Work items: 2D blocks of 64 columns x
// 32 rows, 1D blocks of 2048 points.
struct BRef {
    int32_t dim;
    int32_t nx, ny;
    int32_t pad;
    int64_t ld;
    double wx, wy;   // 1 / hx^2, 1 / hy^2 (1D: wx)
    const double *f;
    double *x;
    float *r32;
    float *e32;
    int64_t item0;   // first work item of this problem
    int64_t nitems;
    int64_t part0;   // first partial slot
};

int64_t ref_items(int dim, int64_t nx, int64_t ny);
// r32 = f - A x (FP64, stored FP32), e32 = 0, partials of ||r||^2 per item
hipError_t launch_batch_ref_resid(const BRef *refs, const int32_t *owner, int64_t nitems, double *part,
                                  hipStream_t st);
// rsq[p] = sum of problem p's partials (fixed order)
hipError_t launch_batch_ref_norm(const BRef *refs, int nref, const double *part, double *rsq,
                                 hipStream_t st);
// x += (double) e32 over the listed items
hipError_t launch_batch_ref_axpy(const BRef *refs, const int32_t *owner, int64_t nitems, hipStream_t st);

bool batch2d_supported(int tx, int ty);
// iso: the work list holds only problems with hx == hy (else only the others)
hipError_t launch_batch_cycle2d(int dt, int tx, int ty, bool iso, const BatchLaunch &L, hipStream_t st);
hipError_t launch_batch_cycle1d(int dt, int t, const BatchLaunch &L, hipStream_t st);
hipError_t launch_batch_judge(const BProb *probs, int nprob, const BCtl *bc, Ctrl *ctrl,
                              const double *part, int64_t npart, hipStream_t st);
hipError_t launch_batch_advance(BCtl *bc, hipStream_t st);
hipError_t launch_batch_init(Ctrl *ctrl, int nprob, BCtl *bc, int64_t max_cycles, hipStream_t st);
hipError_t launch_batch_finalize(int dt, const BProb *probs, int nprob, const Ctrl *ctrl,
                                 hipStream_t st);

int64_t resid2d_mixed_blocks(const Geom2 &g);
hipError_t launch_resid2d_f64_to_f32(const Geom2 &g, const double *f, const double *x, float *r32,
                                     float *e32, double *part, hipStream_t st);
hipError_t launch_axpy_f32_to_f64(const Geom2 &g, const float *e, double *x, hipStream_t st);

}  // namespace hj
