// hj_kernels.hip -- gfx950 kernels for hierarchical and classical Jacobi on the
// 1D 3-point and 2D 5-point Poisson operators (Islam & Wang, arXiv:2006.16465).
//
// Cycle kernels implement the three steps of Sec. 3.3 (2D: Sec. 4.1): one
// workgroup per tile copies the tile and its one-point halo from HBM into LDS,
// runs s Jacobi sub-iterations on the interior with the halo frozen (two LDS
// buffers, Sec. 3.3 even/odd containers), and writes its owned interior points
// to a second global array.  The residual of the iterate being read is
// computed from the same LDS tile at no extra HBM traffic and reduced
// grid-wide in FP64.
//
// Build with -ffp-contract=off: the update association below is part of the
// result and must not be fused.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "hj_launch.h"
#include "hj_tiles.h"

namespace hj {
namespace {

// ============================================================================
// 2D hierarchical cycle: one workgroup per TX x TY tile, LDS ping-pong.
// Thread t owns column t % TX of the tile and rows t / TX + j * (kNT / TX).
// ============================================================================
template <typename T, int TX, int TY, bool RES, bool ISO>
__global__ __launch_bounds__(kNT) void k_cycle2d(Geom2 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 int s, Red red, double tol)
{
    static_assert(kNT % TX == 0 && (TX * TY) % kNT == 0, "tile/threads mismatch");
    if (RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }

    constexpr int P = TX + 2;          // LDS row pitch, halo column each side
    constexpr int R = TY + 2;          // LDS rows, halo row each side
    constexpr int PER = TX * TY / kNT; // points per thread
    constexpr int RSTEP = kNT / TX;
    __shared__ T buf[2][R * P];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int ey = g.ny < TY ? g.ny : TY;
    const int ex = g.nx < TX ? g.nx : TX;
    const int64_t ld = g.ld;

    // step 1: tile + one-point halo into both buffers (0 outside the domain)
    for (int i = threadIdx.x; i < R * P; i += kNT) {
        const int lr = i / P, lc = i - lr * P;
        const int gr = r0 + lr - 1, gc = c0 + lc - 1;
        T v = T(0);
        if (gr >= 0 && gr < g.ny && gc >= 0 && gc < g.nx) v = xin[(int64_t)gr * ld + gc];
        buf[0][i] = v;
        buf[1][i] = v;
    }

    const int tc = threadIdx.x % TX, tr = threadIdx.x / TX;
    const T hh = T(g.hh), wx = T(g.wx), wy = T(g.wy), dinv = T(g.dinv);
    T fb[PER], val[PER];
    double fr[RES ? PER : 1];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = tr + j * RSTEP;
        T fv = T(0);
        if (r < ey && tc < ex) fv = f[(int64_t)(r0 + r) * ld + c0 + tc];
        fb[j] = ISO ? hh * fv : fv;
        if (RES) fr[RES ? j : 0] = (double)fv;
        val[j] = T(0);
    }
    const int rlo = axis_own_begin(g.ny, TY, g.oy, bi) - r0;
    const int rhi = axis_own_end(g.ny, TY, g.oy, bi, g.nty) - r0;
    const int clo = axis_own_begin(g.nx, TX, g.ox, bj) - c0;
    const int chi = axis_own_end(g.nx, TX, g.ox, bj, g.ntx) - c0;
    const bool col_own = tc >= clo && tc < chi;
    __syncthreads();

    // residual of the incoming iterate over the owned points
    double rsq = 0.0;
    if (RES) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tr + j * RSTEP;
            if (col_own && r >= rlo && r < rhi) {
                const int a = (r + 1) * P + tc + 1;
                const T *b0 = buf[0];
                const double rr = res2(fr[RES ? j : 0], (double)b0[a], (double)b0[a - 1],
                                       (double)b0[a + 1], (double)b0[a - P], (double)b0[a + P],
                                       g.wx, g.wy);
                rsq += rr * rr;
            }
        }
    }

    // step 2: s sub-iterations, halo untouched
    for (int k = 0; k < s; ++k) {
        const T *cur = buf[k & 1];
        T *nxt = buf[(k & 1) ^ 1];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tr + j * RSTEP;
            if (r < ey && tc < ex) {
                const int a = (r + 1) * P + tc + 1;
                const T v = upd2<T, ISO>(fb[j], cur[a - 1], cur[a + 1], cur[a - P], cur[a + P],
                                         wx, wy, dinv);
                nxt[a] = v;
                val[j] = v;
            }
        }
        __syncthreads();
    }

    // step 3: owned interior points back to global memory
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = tr + j * RSTEP;
        if (col_own && r >= rlo && r < rhi) xout[(int64_t)(r0 + r) * ld + c0 + tc] = val[j];
    }

    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// ============================================================================
// 2D hierarchical cycle, register-resident: one workgroup of W wavefronts per
// full tile (tile body in hj_tiles.h), fused residual of the incoming iterate.
// ============================================================================
template <typename T, int C, int R, int W, bool RES, bool ISO>
__global__ __launch_bounds__(64 * W, (min_waves_2d<T, C, R>())) void k_cycle2d_reg(Geom2 g, const T *__restrict__ f,
                                                        const T *__restrict__ xin,
                                                        T *__restrict__ xout, int nsub, Red red,
                                                        double tol)
{
    constexpr int NT = 64 * W;
    if (RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<NT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const double rsq = reg_tile_2d<T, C, R, W, RES, ISO, rotate_rows<T>()>(g, xcd_tile(blockIdx.x, gridDim.x), f, xin,
                                                         xout, nsub);
    if (RES) post_partial<NT>(rsq, red.part_cur);
}

// ============================================================================
// 2D classical sweep (global-memory Jacobi, Sec. 3.2 / 4.2): each thread walks
// down RPT rows of one column, so x is read about once per point; W/E come
// from the cache lines the neighbouring lanes fetch.
// ============================================================================
constexpr int kSBX = 64, kSBY = 4, kSRPT = 8;

template <typename T, bool RES, bool ISO, bool SWEEP>
__global__ __launch_bounds__(kNT) void k_sweep2d(Geom2 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 Red red, double tol)
{
    if (SWEEP && RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const int gx = (g.nx + kSBX - 1) / kSBX;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int by = b / gx, bx = b - by * gx;
    const int c = bx * kSBX + (int)(threadIdx.x % kSBX);
    const int rbeg = (by * kSBY + (int)(threadIdx.x / kSBX)) * kSRPT;
    const int64_t ld = g.ld;
    const T hh = T(g.hh), wx = T(g.wx), wy = T(g.wy), dinv = T(g.dinv);
    double rsq = 0.0;
    if (c < g.nx && rbeg < g.ny) {
        T up = rbeg > 0 ? xin[(int64_t)(rbeg - 1) * ld + c] : T(0);
        T cen = xin[(int64_t)rbeg * ld + c];
#pragma unroll
        for (int i = 0; i < kSRPT; ++i) {
            const int r = rbeg + i;
            if (r < g.ny) {
                const int64_t a = (int64_t)r * ld + c;
                const T dn = r + 1 < g.ny ? xin[a + ld] : T(0);
                const T w = c > 0 ? xin[a - 1] : T(0);
                const T e = c + 1 < g.nx ? xin[a + 1] : T(0);
                const T fv = f[a];
                if (SWEEP) xout[a] = upd2<T, ISO>(ISO ? hh * fv : fv, w, e, up, dn, wx, wy, dinv);
                if (RES) {
                    const double rr = res2((double)fv, (double)cen, (double)w, (double)e,
                                           (double)up, (double)dn, g.wx, g.wy);
                    if (!SWEEP && xout) xout[a] = (T)rr;  // residual kernel: optional r_out
                    rsq += rr * rr;
                }
                up = cen;
                cen = dn;
            }
        }
    }
    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// ============================================================================
// 1D hierarchical cycle (tile group body in hj_tiles.h).
// ============================================================================
template <typename T, int TT, bool RES>
__global__ __launch_bounds__(kNT) void k_cycle1d(Geom1 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 int s, Red red, double tol)
{
    if (RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const double rsq = tiles_1d<T, TT, RES>(g, xcd_tile(blockIdx.x, gridDim.x), f, xin, xout, s);
    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// 1D classical sweep / residual: one point per thread.
template <typename T, bool RES, bool SWEEP>
__global__ __launch_bounds__(kNT) void k_sweep1d(Geom1 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 Red red, double tol)
{
    if (SWEEP && RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const int64_t i = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kNT + threadIdx.x;
    double rsq = 0.0;
    if (i < g.n) {
        const T w = i > 0 ? xin[i - 1] : T(0);
        const T e = i + 1 < g.n ? xin[i + 1] : T(0);
        const T fv = f[i];
        if (SWEEP) xout[i] = upd1<T>(T(g.hh) * fv, w, e);
        if (RES) {
            const double rr = res1((double)fv, (double)xin[i], (double)w, (double)e, g.w1);
            if (!SWEEP && xout) xout[i] = (T)rr;
            rsq += rr * rr;
        }
    }
    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

__global__ void k_ctrl_init(Ctrl *ctrl, double sw_tol, int64_t sw_min_c)
{
    ctrl->r0sq = 0.0;
    ctrl->last_rsq = 0.0;
    ctrl->iter = 0;
    ctrl->done_cycle = -1;
    ctrl->stop_at = INT64_MAX;
    ctrl->status = ST_RUNNING;
    ctrl->pad = 0;
    ctrl->sw_tol = sw_tol;
    ctrl->sw_min_c = sw_min_c;
}

// Judge iterate c from n partials left by the previous kernel (one workgroup).
__global__ __launch_bounds__(kNT) void k_judge(const double *part, int n, Ctrl *ctrl, int64_t c,
                                               double tol)
{
    judge_partials<kNT>(part, n, ctrl, c, tol);
}

// ---------------------------------------------------------------- dispatch
// shapes the LDS kernel provides (full or partial tiles)
constexpr bool lds_shape(int tx, int ty)
{
    return (tx == 16 || tx == 32 || tx == 64) && (ty == 16 || ty == 32 || ty == 64);
}

template <typename T, int TX, int TY>
hipError_t cyc2_reg(const Geom2 &g, int s, bool res, const void *f, const void *xin, void *xout,
                    const Red &red, double tol, hipStream_t st)
{
    using S = RegShape<TX, TY>;
    constexpr int C = S::C, R = S::R, W = S::W;
    const unsigned nb = (unsigned)((int64_t)g.ntx * g.nty);
    const T *F = (const T *)f;
    const T *XI = (const T *)xin;
    T *XO = (T *)xout;
    if (res) {
        if (g.iso) k_cycle2d_reg<T, C, R, W, true, true><<<nb, 64 * W, 0, st>>>(g, F, XI, XO, s, red, tol);
        else k_cycle2d_reg<T, C, R, W, true, false><<<nb, 64 * W, 0, st>>>(g, F, XI, XO, s, red, tol);
    } else {
        if (g.iso) k_cycle2d_reg<T, C, R, W, false, true><<<nb, 64 * W, 0, st>>>(g, F, XI, XO, s, red, tol);
        else k_cycle2d_reg<T, C, R, W, false, false><<<nb, 64 * W, 0, st>>>(g, F, XI, XO, s, red, tol);
    }
    return hipGetLastError();
}

template <typename T, int TX, int TY>
hipError_t cyc2(const Geom2 &g, int s, bool res, const void *f, const void *xin, void *xout,
                const Red &red, double tol, hipStream_t st)
{
    if constexpr (RegShape<TX, TY>::ok) {
        if (g.reg && g.nx >= TX && g.ny >= TY)
            return cyc2_reg<T, TX, TY>(g, s, res, f, xin, xout, red, tol, st);
    }
    if constexpr (lds_shape(TX, TY)) {
        const unsigned nb = (unsigned)((int64_t)g.ntx * g.nty);
        const T *F = (const T *)f;
        const T *XI = (const T *)xin;
        T *XO = (T *)xout;
        if (res) {
            if (g.iso) k_cycle2d<T, TX, TY, true, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, s, red, tol);
            else k_cycle2d<T, TX, TY, true, false><<<nb, kNT, 0, st>>>(g, F, XI, XO, s, red, tol);
        } else {
            if (g.iso) k_cycle2d<T, TX, TY, false, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, s, red, tol);
            else k_cycle2d<T, TX, TY, false, false><<<nb, kNT, 0, st>>>(g, F, XI, XO, s, red, tol);
        }
        return hipGetLastError();
    }
    return hipErrorInvalidValue;  // excluded beforehand by cycle2d_runnable
}

#define HJ_TILES(X)                                                                       \
    X(16, 16) X(16, 32) X(16, 64)                                                         \
    X(32, 16) X(32, 32) X(32, 64) X(32, 128)                                              \
    X(64, 16) X(64, 32) X(64, 64) X(64, 128)                                              \
    X(128, 16) X(128, 32) X(128, 64) X(128, 128)

template <typename T>
hipError_t cyc2_t(const Geom2 &g, int s, bool res, const void *f, const void *xin, void *xout,
                  const Red &red, double tol, hipStream_t st)
{
#define HJ_TILE(a, b)                                                                     \
    if (g.tx == a && g.ty == b) return cyc2<T, a, b>(g, s, res, f, xin, xout, red, tol, st);
    HJ_TILES(HJ_TILE)
#undef HJ_TILE
    return hipErrorInvalidValue;
}

template <typename T, int TT>
hipError_t cyc1(const Geom1 &g, int s, bool res, const void *f, const void *xin, void *xout,
                const Red &red, double tol, hipStream_t st)
{
    const unsigned nb = (unsigned)cycle1d_blocks(g);  // the count the judge sums partials over
    if (res) k_cycle1d<T, TT, true><<<nb, kNT, 0, st>>>(g, (const T *)f, (const T *)xin, (T *)xout, s, red, tol);
    else k_cycle1d<T, TT, false><<<nb, kNT, 0, st>>>(g, (const T *)f, (const T *)xin, (T *)xout, s, red, tol);
    return hipGetLastError();
}

template <typename T>
hipError_t cyc1_t(const Geom1 &g, int s, bool res, const void *f, const void *xin, void *xout,
                  const Red &red, double tol, hipStream_t st)
{
    switch (g.t) {
    case 32: return cyc1<T, 32>(g, s, res, f, xin, xout, red, tol, st);
    case 64: return cyc1<T, 64>(g, s, res, f, xin, xout, red, tol, st);
    case 128: return cyc1<T, 128>(g, s, res, f, xin, xout, red, tol, st);
    case 256: return cyc1<T, 256>(g, s, res, f, xin, xout, red, tol, st);
    case 512: return cyc1<T, 512>(g, s, res, f, xin, xout, red, tol, st);
    case 1024: return cyc1<T, 1024>(g, s, res, f, xin, xout, red, tol, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool cycle2d_supported(int tx, int ty)
{
#define HJ_TILE(a, b) if (tx == a && ty == b) return true;
    HJ_TILES(HJ_TILE)
#undef HJ_TILE
    return false;
}

bool cycle2d_runnable(const Geom2 &g)
{
    if (lds_shape(g.tx, g.ty)) return true;
    // tiles with a 128 extent exist only register-resident, for full tiles
    return g.reg && g.nx >= g.tx && g.ny >= g.ty;
}

bool cycle1d_supported(int t)
{
    return t == 32 || t == 64 || t == 128 || t == 256 || t == 512 || t == 1024;
}

int64_t cycle2d_blocks(const Geom2 &g) { return (int64_t)g.ntx * g.nty; }

int64_t sweep2d_blocks(const Geom2 &g)
{
    const int64_t gx = (g.nx + kSBX - 1) / kSBX;
    const int64_t gy = (g.ny + kSBY * kSRPT - 1) / (kSBY * kSRPT);
    return gx * gy;
}

int64_t resid2d_blocks(const Geom2 &g) { return sweep2d_blocks(g); }

int64_t cycle1d_blocks(const Geom1 &g)
{
    const int64_t G = tiles_per_block_1d(g.t);
    return (g.nt + G - 1) / G;
}

int64_t sweep1d_blocks(const Geom1 &g) { return (g.n + kNT - 1) / kNT; }
int64_t resid1d_blocks(const Geom1 &g) { return sweep1d_blocks(g); }

hipError_t launch_cycle2d(int dt, const Geom2 &g, int s, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st)
{
    if (dt == F64) return cyc2_t<double>(g, s, res, f, xin, xout, red, tol, st);
    return cyc2_t<float>(g, s, res, f, xin, xout, red, tol, st);
}

template <typename T>
static hipError_t sw2(const Geom2 &g, bool res, const void *f, const void *xin, void *xout,
                      const Red &red, double tol, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep2d_blocks(g);
    const T *F = (const T *)f;
    const T *XI = (const T *)xin;
    T *XO = (T *)xout;
    if (res) {
        if (g.iso) k_sweep2d<T, true, true, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, red, tol);
        else k_sweep2d<T, true, false, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, red, tol);
    } else {
        if (g.iso) k_sweep2d<T, false, true, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, red, tol);
        else k_sweep2d<T, false, false, true><<<nb, kNT, 0, st>>>(g, F, XI, XO, red, tol);
    }
    return hipGetLastError();
}

hipError_t launch_sweep2d(int dt, const Geom2 &g, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st)
{
    if (dt == F64) return sw2<double>(g, res, f, xin, xout, red, tol, st);
    return sw2<float>(g, res, f, xin, xout, red, tol, st);
}

hipError_t launch_resid2d(int dt, const Geom2 &g, const void *f, const void *x, void *r_out,
                          double *part, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep2d_blocks(g);
    const Red red{part, nullptr, nullptr, 0, 0};
    if (dt == F64)
        k_sweep2d<double, true, true, false><<<nb, kNT, 0, st>>>(
            g, (const double *)f, (const double *)x, (double *)r_out, red, -1.0);
    else
        k_sweep2d<float, true, true, false><<<nb, kNT, 0, st>>>(
            g, (const float *)f, (const float *)x, (float *)r_out, red, -1.0);
    return hipGetLastError();
}

hipError_t launch_cycle1d(int dt, const Geom1 &g, int s, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st)
{
    if (dt == F64) return cyc1_t<double>(g, s, res, f, xin, xout, red, tol, st);
    return cyc1_t<float>(g, s, res, f, xin, xout, red, tol, st);
}

hipError_t launch_sweep1d(int dt, const Geom1 &g, bool res, const void *f, const void *xin,
                          void *xout, const Red &red, double tol, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep1d_blocks(g);
    if (dt == F64) {
        if (res) k_sweep1d<double, true, true><<<nb, kNT, 0, st>>>(g, (const double *)f, (const double *)xin, (double *)xout, red, tol);
        else k_sweep1d<double, false, true><<<nb, kNT, 0, st>>>(g, (const double *)f, (const double *)xin, (double *)xout, red, tol);
    } else {
        if (res) k_sweep1d<float, true, true><<<nb, kNT, 0, st>>>(g, (const float *)f, (const float *)xin, (float *)xout, red, tol);
        else k_sweep1d<float, false, true><<<nb, kNT, 0, st>>>(g, (const float *)f, (const float *)xin, (float *)xout, red, tol);
    }
    return hipGetLastError();
}

hipError_t launch_resid1d(int dt, const Geom1 &g, const void *f, const void *x, void *r_out,
                          double *part, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep1d_blocks(g);
    const Red red{part, nullptr, nullptr, 0, 0};
    if (dt == F64)
        k_sweep1d<double, true, false><<<nb, kNT, 0, st>>>(g, (const double *)f, (const double *)x, (double *)r_out, red, -1.0);
    else
        k_sweep1d<float, true, false><<<nb, kNT, 0, st>>>(g, (const float *)f, (const float *)x, (float *)r_out, red, -1.0);
    return hipGetLastError();
}

hipError_t launch_judge(const double *part, int n, Ctrl *ctrl, int64_t c, double tol, hipStream_t st)
{
    k_judge<<<1, kNT, 0, st>>>(part, n, ctrl, c, tol);
    return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl *ctrl, hipStream_t st, double sw_tol, int64_t sw_min_c)
{
    k_ctrl_init<<<1, 1, 0, st>>>(ctrl, sw_tol, sw_min_c);
    return hipGetLastError();
}

}  // namespace hj
