// hj_batch.hip -- many independent problems (2D and 1D, uneven sizes) solved
// together: one launch per cycle covers the work list of every problem.
//
// Each step (a fixed launch sequence, so a captured graph can replay it):
//   k_batch_cycle2d  every 2D tile of every running problem (one launch for
//                    problems with hx == hy, one for the rest): one cycle of
//                    Sec. 4.1 on the problem's current phase, from its
//                    iterate j into the other buffer, the residual of
//                    iterate j fused into the load (per-tile partials);
//   k_batch_cycle1d  the same for the 1D tile groups (Sec. 3.3);
//   k_batch_cycle_vc the same for variable-coefficient 2D problems (the
//                    right-hand sides of one diffusion operator);
//   k_batch_judge    per problem, the partials in a fixed order, the verdict
//                    on iterate j, and the next phase.
// Every problem carries its own iterate index and buffer selectors, so
// problems move through their phases independently: no step waits for
// another problem.  A plain batch has one phase (MAIN): a problem that stops
// at iterate j keeps it in buffer j & 1 (the verdict lands before the next
// cycle), so two buffers per problem suffice, and the tile bodies are the
// single-problem ones (hj_tiles.h): iterates equal those of each problem's own
// solve bit for bit.
//
// Refined batches (FP64 problems): MAIN FP64 cycles until the switch, then
// refinement steps (REF, run by the problem's work items in place of a
// cycle): x <- x + e and r = f - A x in FP64 in one pass (r stored FP32, the
// next correction buffer cleared), FP32 cycles on A e = r from e = 0 (INNER)
// to a per-problem target, and again, until the FP64 residual meets the
// tolerance.  One kernel per tile kind holds the three bodies, so a step
// launches each work item once whatever its problem's phase.  The FP32 floor of
// a problem is predicted as F = 2 u s / -ln(rho) (u = 2^-24, rho the
// per-cycle residual factor measured before the switch: rounding of order
// u |x| in every sweep sets the residual FP32 Jacobi can reach, relative to
// the slowest modes' eigenvalue).  A problem switches once one correction
// solve stopped at 4F or above can finish it (relative residual <= tol / 8F,
// and <= switch_tol); the target of a correction solve is the larger of
// inner_min, what the outer tolerance still needs (with a factor 2 to spare)
// and 2F.  A problem with F above fmax stays in FP64; a correction solve that
// stops halving its residual (within 8 + 4 halving times of the measured
// rate) is applied and the problem continues in FP64.
//
// One workgroup per work item, handed out XCD by XCD in list order (problems
// in turn, tiles row-major), rather than a grid-stride loop over the list:
// the loop kept about 30 more VGPRs live around the tile body (154 against
// 124 at 64x64 FP64), one wave per SIMD fewer.  Items of problems that have
// stopped, or are in a phase of the other precision, return after reading
// the problem's state.
#include <hip/hip_runtime.h>

#include "hj_launch.h"
#include "hj_tiles.h"
#include "hj_vc_tile.h"

namespace hj {
namespace {

constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff
constexpr double kLn2 = 0.6931471805599453;

template <int NT>
__device__ __forceinline__ void post_partial_at(double mine, double *slot)
{
    __shared__ double red[NT / 64];
    const double bs = block_sum<NT>(mine, red);
    if (threadIdx.x == 0) *slot = bs;
}

constexpr int kRBX = 64, kRRPT = 8;  // refinement-step 2D blocks: 64 columns x (4 x 8) rows
constexpr int kR1 = 2048;           // refinement-step 1D blocks

__device__ __forceinline__ double xpe(const double *x, const float *e, int64_t a)
{
    return e ? x[a] + (double)e[a] : x[a];
}

// Buffers of the main cycle (iterate j of the main phase from buffer
// xsel ^ (j & 1) into the other) and of the inner one (correction e_j).
template <typename T>
__device__ __forceinline__ void main_arrays(const BProb &P, const BState &S, const T *&xin, T *&xout)
{
    const int b = S.xsel ^ (int)(S.j & 1);
    xin = (const T *)(b ? P.s1 : P.x);
    xout = (T *)(b ? P.x : P.s1);
}

__device__ __forceinline__ void inner_arrays(const BProb &P, const BState &S, const float *&ein, float *&eout)
{
    const int b = S.esel ^ (int)(S.j & 1);
    ein = b ? P.e1 : P.e0;
    eout = b ? P.e0 : P.e1;
}

template <int NT>
__device__ double ref_blocks(const BProb &P, const BState &S, int64_t item, int64_t nitems);

// Batch modes: plain FP64, plain FP32, refined (each work item runs its
// problem's phase: an FP64 main cycle, an FP32 inner cycle, or its share of a
// refinement step).
enum : int { BM_F64 = 0, BM_F32 = 1, BM_REF = 2 };

template <int M, int C, int R, int W, bool ISO>
__global__ __launch_bounds__(64 * W, (min_waves_2d<std::conditional_t<M == BM_F32, float, double>, C, R>()))
void k_batch_cycle2d(const BProb *__restrict__ probs,
                                                          const int32_t *__restrict__ owner,
                                                          int64_t nitems, const BState *__restrict__ state,
                                                          double *part, int s)
{
    constexpr int NT = 64 * W;
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const int p = owner[w];
    const BState &S = state[p];
    if (S.status != ST_RUNNING) return;
    const BProb &P = probs[p];
    const int tile = (int)(w - P.item0);
    double rsq;
    if (M == BM_F32) {
        const float *xin;
        float *xout;
        main_arrays<float>(P, S, xin, xout);
        rsq = reg_tile_2d<float, C, R, W, true, ISO, rotate_rows<float>()>(P.g2, tile, (const float *)P.f, xin,
                                                                          xout, s);
    } else if (M == BM_F64) {
        const double *xin;
        double *xout;
        main_arrays<double>(P, S, xin, xout);
        rsq = reg_tile_2d<double, C, R, W, true, ISO, rotate_rows<double>()>(P.g2, tile, (const double *)P.f,
                                                                            xin, xout, s);
    } else if (S.phase == PH_MAIN) {
        // refined: both precisions share one LDS pool sized for FP64
        const double *xin;
        double *xout;
        main_arrays<double>(P, S, xin, xout);
        rsq = reg_tile_2d<double, C, R, W, true, ISO, rotate_rows<double>(), 8>(P.g2, tile, (const double *)P.f,
                                                                               xin, xout, s);
    } else if (S.phase == PH_INNER) {
        const float *ein;
        float *eout;
        inner_arrays(P, S, ein, eout);
        rsq = reg_tile_2d<float, C, R, W, true, ISO, rotate_rows<float>(), 8>(P.g2, tile, P.r32, ein, eout, s);
    } else {
        rsq = ref_blocks<NT>(P, S, tile, P.nitems);
    }
    post_partial_at<NT>(rsq, &part[P.part0 + tile]);
}

template <int M, int TT>
__global__ __launch_bounds__(kNT) void k_batch_cycle1d(const BProb *__restrict__ probs,
                                                       const int32_t *__restrict__ owner,
                                                       int64_t nitems, const BState *__restrict__ state,
                                                       double *part, int s)
{
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const int p = owner[w];
    const BState &S = state[p];
    if (S.status != ST_RUNNING) return;
    const BProb &P = probs[p];
    const int64_t blk = w - P.item0;
    double rsq;
    if (M == BM_F32) {
        const float *xin;
        float *xout;
        main_arrays<float>(P, S, xin, xout);
        rsq = tiles_1d<float, TT, true>(P.g1, blk, (const float *)P.f, xin, xout, s);
    } else if (M == BM_F64 || S.phase == PH_MAIN) {
        const double *xin;
        double *xout;
        main_arrays<double>(P, S, xin, xout);
        rsq = tiles_1d<double, TT, true>(P.g1, blk, (const double *)P.f, xin, xout, s);
    } else if (S.phase == PH_INNER) {
        const float *ein;
        float *eout;
        inner_arrays(P, S, ein, eout);
        rsq = tiles_1d<float, TT, true>(P.g1, blk, P.r32, ein, eout, s);
    } else {
        rsq = ref_blocks<kNT>(P, S, blk, P.nitems);
    }
    post_partial_at<kNT>(rsq, &part[P.part0 + blk]);
}

// Variable-coefficient 2D problems (dim 3, FP64, plain): the tile bodies of
// the single-problem kernel (hj_vc_tile.h).
template <int TX, int TY>
__global__ __launch_bounds__((vc_threads<TX, TY>())) void k_batch_cycle_vc(const BProb *__restrict__ probs,
                                                        const int32_t *__restrict__ owner, int64_t nitems,
                                                        const BState *__restrict__ state, double *part, int s)
{
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const int p = owner[w];
    const BState &S = state[p];
    if (S.status != ST_RUNNING) return;
    const BProb &P = probs[p];
    const double *xin;
    double *xout;
    main_arrays<double>(P, S, xin, xout);
    const int tile = (int)(w - P.item0);
    const double rsq = tile_vc<TX, TY, true>(P.gv, tile, (const double *)P.f, xin, xout, s);
    post_partial_at<vc_threads<TX, TY>()>(rsq, &part[P.part0 + tile]);
}

// ---------------------------------------------------------------- judge
__device__ __forceinline__ void stop(BState &t, int32_t status, int buf, int64_t add)
{
    t.status = status;
    t.xsel = buf;
    t.used += add;
}

// Refinement step on x in main buffer rx with the correction in inner buffer
// esrc (-1: none): the new x goes to the other main buffer (stays put without
// a correction), the next correction solve starts in the inner buffer that
// does not hold e.
__device__ __forceinline__ void begin_ref(BState &t, int rx, int esrc, int32_t next)
{
    t.rx = rx;
    t.esrc = esrc;
    t.xsel = esrc >= 0 ? rx ^ 1 : rx;
    t.esel = esrc >= 0 ? esrc ^ 1 : 0;
    t.j = 0;
    t.phase = PH_REF;
    t.next = next;
}

__device__ __forceinline__ double fp32_floor(const BProb &P, double lnrate)
{
    return lnrate < 0.0 ? 2.0 * kU32 * (double)P.s / -lnrate : 0.0;
}

// MAIN of a refined problem below switch_tol: switch to FP32 corrections
// now?  The per-cycle rate (since the residual passed 10 switch_tol, else over
// the last cycle) predicts the FP32 floor F.  One correction solve stopped at
// 4F or above stays clear of it and of the slow-mode error that FP32 rounding
// plants as it nears it, so the switch waits until such a solve finishes the
// job: relative residual <= tol / (8F) (the solve then asks for
// tol / (2 rel) >= 4F).  Problems with F > fmax stay in FP64.
__device__ __forceinline__ bool switch_now(const BProb &P, BState &t, double acc, double prev, double rel,
                                           const BRefine &rf)
{
    const int64_t j = t.j;
    double lr = 0.0;
    if (t.mark_j >= 0 && j > t.mark_j) lr = 0.5 * log(acc / t.mark_rsq) / (double)(j - t.mark_j);
    else if (j > 0 && prev > 0.0) lr = 0.5 * log(acc / prev);
    const double F = fp32_floor(P, lr);
    if (F > rf.fmax) return false;
    if (F > 0.0 && rel > P.tol / (8.0 * F)) return false;
    t.lnrate = lr;
    return true;
}

// Lane 0 of the problem's wavefront.  acc: sum of the partials of this step
// (the cycle's residual of iterate j, or the refinement step's FP64
// residual of the new x).
__device__ void judge_problem(const BProb &P, BState &t, double acc, const BRefine &rf)
{
    const double tol = P.tol;
    switch (t.phase) {
    case PH_MAIN: {
        const int64_t j = t.j;
        if (j == 0 && t.used == 0) t.r0sq = acc;
        const double prev = t.rsq;
        t.rsq = acc;
        const double rel = t.r0sq > 0.0 ? sqrt(acc) / sqrt(t.r0sq) : 0.0;
        const int here = t.xsel ^ (int)(j & 1);
        if (!isfinite(acc)) {
            stop(t, ST_NONFINITE, here, j);
        } else if (rel <= tol) {
            stop(t, ST_CONVERGED, here, j);
        } else if (t.used + j >= P.max_cycles) {
            stop(t, ST_LIMIT, here, j);
        } else if (rf.refine && !t.cont && rel <= rf.switch_tol && switch_now(P, t, acc, prev, rel, rf)) {
            // hand over iterate j + 1: the cycle that evaluated iterate j wrote it
            t.used += j + 1;
            begin_ref(t, t.xsel ^ (int)((j + 1) & 1), -1, PH_INNER);
        } else {
            if (rf.refine && !t.cont && t.mark_j < 0 && rel <= 10.0 * rf.switch_tol) {
                t.mark_rsq = acc;
                t.mark_j = j;
            }
            t.j = j + 1;
        }
        break;
    }
    case PH_REF: {
        t.rsq = acc;
        const double rel = t.r0sq > 0.0 ? sqrt(acc) / sqrt(t.r0sq) : 0.0;
        if (!isfinite(acc)) {
            stop(t, ST_NONFINITE, t.xsel, 0);
        } else if (rel <= tol) {
            stop(t, ST_CONVERGED, t.xsel, 0);
        } else if (t.next == PH_END || t.used >= P.max_cycles) {
            stop(t, ST_LIMIT, t.xsel, 0);
        } else if (t.next == PH_MAIN || t.outer >= rf.max_outer) {
            // FP64 cycles from the new x on
            t.cont = 1;
            t.j = 0;
            t.phase = PH_MAIN;
        } else {
            const double need = 0.5 * tol * sqrt(t.r0sq) / sqrt(acc);
            const double want = fmax(fmax(rf.inner_min, need), 2.0 * fp32_floor(P, t.lnrate));
            t.in_tolsq = want * want * acc;
            t.outer += 1;
            t.mark_rsq = acc;
            t.mark_j = 0;
            t.j = 0;
            t.phase = PH_INNER;
        }
        break;
    }
    case PH_INNER: {
        const int64_t j = t.j;
        // the latest correction e_{j+1} (written by the cycle that evaluated
        // e_j) unless the budget ends at e_j
        const int64_t take = t.used + j + 1 <= P.max_cycles ? j + 1 : j;
        if (!isfinite(acc)) {
            // an FP32 correction that overflowed is dropped; FP64 from x on
            begin_ref(t, t.xsel, -1, PH_MAIN);
        } else if (acc <= t.in_tolsq) {
            t.used += take;
            begin_ref(t, t.xsel, t.esel ^ (int)(take & 1), PH_INNER);
        } else if (t.used + j >= P.max_cycles) {
            t.used += j;
            begin_ref(t, t.xsel, t.esel ^ (int)(j & 1), PH_END);
        } else {
            bool stalled = false;
            if (acc <= 0.25 * t.mark_rsq) {
                t.mark_rsq = acc;
                t.mark_j = j;
            } else {
                const double win = t.lnrate < 0.0 ? 8.0 + 4.0 * kLn2 / -t.lnrate : 32.0;
                stalled = (double)(j - t.mark_j) > win;
            }
            if (stalled) {
                t.used += take;
                begin_ref(t, t.xsel, t.esel ^ (int)(take & 1), PH_MAIN);
            } else {
                t.j = j + 1;
            }
        }
        break;
    }
    default:
        break;
    }
}

__device__ __forceinline__ double sum_parts(const double *base, int64_t n, int lane)
{
    double acc = 0.0;
    for (int64_t i = lane; i < n; i += 64) acc += base[i];
    return wave_sum(acc);
}

// One wavefront per problem: partials summed lane-strided in index order,
// then a fixed butterfly; lane 0 updates the state.
__global__ __launch_bounds__(256) void k_batch_judge(const BProb *__restrict__ probs, int nprob,
                                                     BState *state, const double *part, BRefine rf)
{
    const int lane = (int)threadIdx.x & 63;
    const int p = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    if (p >= nprob) return;
    if (state[p].status != ST_RUNNING) return;
    const BProb &P = probs[p];
    const double acc = sum_parts(part + P.part0, P.nitems, lane);
    if (lane == 0) {
        BState t = state[p];
        judge_problem(P, t, acc, rf);
        state[p] = t;
    }
}

__global__ __launch_bounds__(256) void k_batch_init(BState *state, int nprob)
{
    for (int p = (int)(blockIdx.x * blockDim.x + threadIdx.x); p < nprob; p += (int)(gridDim.x * blockDim.x)) {
        BState t{};
        t.mark_j = -1;
        t.esrc = -1;
        t.status = ST_RUNNING;
        t.phase = PH_MAIN;
        state[p] = t;
    }
}

// Main buffer holding a problem's result (a problem still running: its
// latest judged main iterate, or its refined x).
__device__ __forceinline__ int result_buf(const BState &S)
{
    if (S.status == ST_RUNNING && S.phase == PH_MAIN && S.j > 0) return S.xsel ^ (int)((S.j - 1) & 1);
    if (S.status == ST_RUNNING && S.phase == PH_REF) return S.rx;
    return S.xsel;
}

// Grid: (problem, chunk).
__global__ __launch_bounds__(256) void k_batch_finalize(const BProb *__restrict__ probs,
                                                        const BState *state)
{
    const int p = (int)blockIdx.x;
    if (result_buf(state[p]) != 1) return;
    const BProb &P = probs[p];
    const int64_t nx = P.dim == 2 ? P.g2.nx : P.dim == 3 ? P.gv.nx : P.g1.n;
    const int64_t ny = P.dim == 2 ? P.g2.ny : P.dim == 3 ? P.gv.ny : 1;
    const int64_t ld = P.dim == 2 ? P.g2.ld : P.dim == 3 ? P.gv.ld : P.g1.n;
    const int64_t total = nx * ny;
    for (int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.y * 256) {
        const int64_t r = i / nx, q = i - r * nx;
        const int64_t a = r * ld + q;
        if (P.dt == F64) ((double *)P.x)[a] = ((const double *)P.s1)[a];
        else ((float *)P.x)[a] = ((const float *)P.s1)[a];
    }
}

// ---------------------------------------------------------------- refinement step
// y = x + e (FP64; y = x without a correction) written to the new main
// buffer, r = f - A y in FP64 (the oracle's residual association) stored
// FP32, the next correction buffer cleared; this thread's share of ||r||^2.
// Every point's y is formed the same way by whichever thread reads it.
// Blocks: 2D 64 columns x 32 rows (a thread per column and 8-row group),
// 1D 2048 points; work item `item` of nitems takes blocks item, item +
// nitems, ...
template <int NT>
__device__ double ref_blocks(const BProb &P, const BState &S, int64_t item, int64_t nitems)
{
    const double *f = (const double *)P.f;
    const double *x = (const double *)(S.rx ? P.s1 : P.x);
    double *xd = (double *)(S.xsel ? P.s1 : P.x);
    const float *e = S.esrc < 0 ? nullptr : (S.esrc ? P.e1 : P.e0);
    float *ez = S.esel ? P.e1 : P.e0;
    float *r32 = P.r32;
    double rsq = 0.0;
    for (int64_t blk = item; blk < P.rnitems; blk += nitems) {
        if (P.dim == 2) {
            const Geom2 &g = P.g2;
            const int gx = (g.nx + kRBX - 1) / kRBX;
            const int by = (int)(blk / gx), bx = (int)(blk - (int64_t)by * gx);
            const int c = bx * kRBX + (int)(threadIdx.x % kRBX);
            if (c >= g.nx) continue;
            const int64_t ld = g.ld;
            for (int grp = (int)(threadIdx.x / kRBX); grp < 4; grp += NT / kRBX) {
                const int rbeg = (by * 4 + grp) * kRRPT;
                if (rbeg >= g.ny) break;
                double up = rbeg > 0 ? xpe(x, e, (int64_t)(rbeg - 1) * ld + c) : 0.0;
                double cen = xpe(x, e, (int64_t)rbeg * ld + c);
                for (int i = 0; i < kRRPT; ++i) {
                    const int r = rbeg + i;
                    if (r >= g.ny) break;
                    const int64_t a = (int64_t)r * ld + c;
                    const double dn = r + 1 < g.ny ? xpe(x, e, a + ld) : 0.0;
                    const double wv = c > 0 ? xpe(x, e, a - 1) : 0.0;
                    const double ev = c + 1 < g.nx ? xpe(x, e, a + 1) : 0.0;
                    const double rr = res2(f[a], cen, wv, ev, up, dn, g.wx, g.wy);
                    if (e) xd[a] = cen;
                    r32[a] = (float)rr;
                    ez[a] = 0.0f;
                    rsq += rr * rr;
                    up = cen;
                    cen = dn;
                }
            }
        } else {
            const Geom1 &g = P.g1;
            const int64_t n = g.n;
            for (int64_t i = blk * kR1 + threadIdx.x; i < std::min(n, (blk + 1) * kR1); i += NT) {
                const double y = xpe(x, e, i);
                const double wv = i > 0 ? xpe(x, e, i - 1) : 0.0;
                const double ev = i + 1 < n ? xpe(x, e, i + 1) : 0.0;
                const double rr = res1(f[i], y, wv, ev, g.w1);
                if (e) xd[i] = y;
                r32[i] = (float)rr;
                ez[i] = 0.0f;
                rsq += rr * rr;
            }
        }
    }
    return rsq;
}

// ---------------------------------------------------------------- dispatch
template <int M, int TX, int TY, bool ISO>
hipError_t bcyc2(const BatchLaunch &L, hipStream_t st)
{
    using S = RegShape<TX, TY>;
    k_batch_cycle2d<M, S::C, S::R, S::W, ISO><<<(unsigned)L.nitems, 64 * S::W, 0, st>>>(
        L.probs, L.owner, L.nitems, L.state, L.part, L.s);
    return hipGetLastError();
}

template <int M, int TT>
hipError_t bcyc1(const BatchLaunch &L, hipStream_t st)
{
    k_batch_cycle1d<M, TT><<<(unsigned)L.nitems, kNT, 0, st>>>(L.probs, L.owner, L.nitems, L.state, L.part,
                                                               L.s);
    return hipGetLastError();
}

#define HJ_BATCH_TILES2(X) X(32, 16) X(32, 32) X(32, 64) X(32, 128) X(64, 16) X(64, 32) X(64, 64) X(64, 128)

template <int M>
hipError_t bcyc2_m(int tx, int ty, bool iso, const BatchLaunch &L, hipStream_t st)
{
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return iso ? bcyc2<M, a, b, true>(L, st) : bcyc2<M, a, b, false>(L, st);
    HJ_BATCH_TILES2(HJ_TILE)
#undef HJ_TILE
    return hipErrorInvalidValue;
}

template <int M>
hipError_t bcyc1_m(int t, const BatchLaunch &L, hipStream_t st)
{
    switch (t) {
    case 32: return bcyc1<M, 32>(L, st);
    case 64: return bcyc1<M, 64>(L, st);
    case 128: return bcyc1<M, 128>(L, st);
    case 256: return bcyc1<M, 256>(L, st);
    case 512: return bcyc1<M, 512>(L, st);
    case 1024: return bcyc1<M, 1024>(L, st);
    default: return hipErrorInvalidValue;
    }
}

template <int TX, int TY>
hipError_t bcycvc(const BatchLaunch &L, hipStream_t st)
{
    k_batch_cycle_vc<TX, TY><<<(unsigned)L.nitems, vc_threads<TX, TY>(), 0, st>>>(L.probs, L.owner, L.nitems,
                                                                                  L.state, L.part, L.s);
    return hipGetLastError();
}

}  // namespace

bool batch_vc_supported(int tx, int ty)
{
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return true;
    HJ_VC_TILES(HJ_TILE)
#undef HJ_TILE
    return false;
}

hipError_t launch_batch_cycle_vc(int tx, int ty, const BatchLaunch &L, hipStream_t st)
{
    if (L.nitems <= 0) return hipSuccess;
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return bcycvc<a, b>(L, st);
    HJ_VC_TILES(HJ_TILE)
#undef HJ_TILE
    return hipErrorInvalidValue;
}

int64_t ref_items(int dim, int64_t nx, int64_t ny)
{
    if (dim == 2) return ((nx + kRBX - 1) / kRBX) * ((ny + 4 * kRRPT - 1) / (4 * kRRPT));
    return (nx + kR1 - 1) / kR1;
}

bool batch2d_supported(int tx, int ty)
{
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return true;
    HJ_BATCH_TILES2(HJ_TILE)
#undef HJ_TILE
    return false;
}

hipError_t launch_batch_cycle2d(int dt, bool refine, int tx, int ty, bool iso, const BatchLaunch &L,
                                hipStream_t st)
{
    if (L.nitems <= 0) return hipSuccess;
    if (refine) return bcyc2_m<BM_REF>(tx, ty, iso, L, st);
    return dt == F64 ? bcyc2_m<BM_F64>(tx, ty, iso, L, st) : bcyc2_m<BM_F32>(tx, ty, iso, L, st);
}

hipError_t launch_batch_cycle1d(int dt, bool refine, int t, const BatchLaunch &L, hipStream_t st)
{
    if (L.nitems <= 0) return hipSuccess;
    if (refine) return bcyc1_m<BM_REF>(t, L, st);
    return dt == F64 ? bcyc1_m<BM_F64>(t, L, st) : bcyc1_m<BM_F32>(t, L, st);
}

hipError_t launch_batch_judge(const BProb *probs, int nprob, BState *state, const double *part,
                              const BRefine &rf, hipStream_t st)
{
    k_batch_judge<<<(unsigned)((nprob + 3) / 4), 256, 0, st>>>(probs, nprob, state, part, rf);
    return hipGetLastError();
}

hipError_t launch_batch_init(BState *state, int nprob, hipStream_t st)
{
    const unsigned nb = (unsigned)((nprob + 255) / 256);
    k_batch_init<<<nb > 0 ? nb : 1, 256, 0, st>>>(state, nprob);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BProb *probs, int nprob, const BState *state, hipStream_t st)
{
    const dim3 grid((unsigned)nprob, 16);
    k_batch_finalize<<<grid, 256, 0, st>>>(probs, state);
    return hipGetLastError();
}

}  // namespace hj
