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

namespace hj {
namespace {

// ---------------------------------------------------------------- updates
// 2D: iso  -> (h^2 f + ((W + E) + (S + N))) * 0.25      (Sec. 4.2, dx == dy)
//     else -> (f + (wx (W + E) + wy (S + N))) * dinv    (Sec. 4.2 general form)
template <typename T, bool ISO>
__device__ __forceinline__ T upd2(T b, T w, T e, T s, T n, T wx, T wy, T dinv)
{
    if (ISO) return (b + ((w + e) + (s + n))) * T(0.25);
    return (b + (wx * (w + e) + wy * (s + n))) * dinv;
}

// 1D: (h^2 f + (W + E)) * 0.5                            (Sec. 3.4)
template <typename T>
__device__ __forceinline__ T upd1(T bh, T w, T e)
{
    return (bh + (w + e)) * T(0.5);
}

// r = f - A x in FP64
__device__ __forceinline__ double res2(double f, double x, double w, double e, double s, double n,
                                       double wx, double wy)
{
    return f - (wx * ((2.0 * x - w) - e) + wy * ((2.0 * x - s) - n));
}

__device__ __forceinline__ double res1(double f, double x, double w, double e, double w1)
{
    return f - w1 * ((2.0 * x - w) - e);
}

constexpr int kNT = 256;  // threads per workgroup of every kernel here

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
        if (read_status(red.ctrl) != ST_RUNNING) return;
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
// 2D hierarchical cycle, register-resident.  A workgroup of W wavefronts takes
// one full tile of TX = 16*C columns by TY = 4*R*W rows.  Thread t belongs to
// row group k = t / 16 (4 per wavefront, NG = 4W in all) and lane j = t % 16
// of that group, and holds rows [kR, kR + R) x columns [jC, jC + C) of the
// tile in VGPRs, so a 16-lane DPP row spans the whole tile width.
// x-neighbours in other lanes come from DPP row shifts; y-neighbours in other
// row groups through LDS interface rows, double-buffered so that one barrier
// per sweep suffices.  The frozen halo sits in registers (columns -1 and TX,
// in the first / last lane of each DPP row) and in LDS (rows -1 and TY).
// Used when the grid holds at least one full tile in each direction.
//
// Isotropic update in FMA form: fma(S, 1/4, h^2 f / 4) with S = (W + E) +
// (S + N) equals (h^2 f + S) * 1/4 rounded the two-step way, because scaling
// by a power of two commutes with rounding; this holds whenever the values
// involved are normal numbers (magnitudes above 2^-1020 in FP64, 2^-124 in
// FP32).
// ============================================================================
constexpr int kDppRowShr1 = 0x111;  // lane i <- lane i - 1 of its 16-lane row
constexpr int kDppRowShl1 = 0x101;  // lane i <- lane i + 1 of its 16-lane row

// Lanes whose source falls outside the 16-lane row receive 0 (bound_ctrl).
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}

// s * 1/4 + b with one rounding, in the three-address VOP3 form (the compiler's
// two-address v_fmac would first copy b, which stays live across sweeps)
// (0.25 is not an inline constant and VOP3 takes no literal: it rides in SGPRs)
__device__ __forceinline__ double fma_quarter(double sv, double b)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(sv), "s"(0.25), "v"(b));
    return r;
}

__device__ __forceinline__ float fma_quarter(float sv, float b)
{
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(sv), "s"(0.25f), "v"(b));
    return r;
}

template <typename T, int C, int R, int W, bool RES, bool ISO>
__global__ __launch_bounds__(64 * W) void k_cycle2d_reg(Geom2 g, const T *__restrict__ f,
                                                        const T *__restrict__ xin,
                                                        T *__restrict__ xout, int nsub, Red red,
                                                        double tol)
{
    constexpr int TX = 16 * C, TY = 4 * R * W, NG = 4 * W, NT = 64 * W;
    if (RES) {
        if (read_status(red.ctrl) != ST_RUNNING) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<NT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    __shared__ T s_top[2][NG][TX];  // first row of each row group, by sweep parity
    __shared__ T s_bot[2][NG][TX];  // last row of each row group
    __shared__ T s_halo[2][TX];     // frozen rows -1 and TY

    const int k = (int)threadIdx.x >> 4, j = (int)threadIdx.x & 15;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int64_t ld = g.ld;
    const int lr0 = k * R, lc0 = j * C;
    const int64_t base = (int64_t)(r0 + lr0) * ld + c0 + lc0;

    // step 1: tile, halo and f into registers / LDS
    T x[R][C], bq[R][C], hw[R], he[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            x[i][c] = xin[base + (int64_t)i * ld + c];
            bq[i][c] = f[base + (int64_t)i * ld + c];  // f for now, scaled after the residual
        }
        hw[i] = (j == 0 && c0 > 0) ? xin[base + (int64_t)i * ld - 1] : T(0);
        he[i] = (j == 15 && c0 + TX < g.nx) ? xin[base + (int64_t)i * ld + C] : T(0);
    }
    if (k == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_halo[0][lc0 + c] = r0 > 0 ? xin[(int64_t)(r0 - 1) * ld + c0 + lc0 + c] : T(0);
    }
    if (k == NG - 1) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_halo[1][lc0 + c] =
                r0 + TY < g.ny ? xin[(int64_t)(r0 + TY) * ld + c0 + lc0 + c] : T(0);
    }
    const int rlo = axis_own_begin(g.ny, TY, g.oy, bi) - r0 - lr0;
    const int rhi = axis_own_end(g.ny, TY, g.oy, bi, g.nty) - r0 - lr0;
    const int clo = axis_own_begin(g.nx, TX, g.ox, bj) - c0 - lc0;
    const int chi = axis_own_end(g.nx, TX, g.ox, bj, g.ntx) - c0 - lc0;

    const T wx = T(g.wx), wy = T(g.wy), dinv = T(g.dinv);
    T up[C], dn[C];
    // Publish this group's first / last rows for the sweep of parity par and
    // fetch the neighbouring groups' (or the frozen halo rows).  A buffer is
    // rewritten two sweeps later, after a barrier that every thread reaches
    // only once its reads from it are done.
    auto exchange = [&](int par) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s_top[par][k][lc0 + c] = x[0][c];
            s_bot[par][k][lc0 + c] = x[R - 1][c];
        }
        __syncthreads();
        const T *pu = k == 0 ? &s_halo[0][lc0] : &s_bot[par][k - 1][lc0];
        const T *pd = k == NG - 1 ? &s_halo[1][lc0] : &s_top[par][k + 1][lc0];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            up[c] = pu[c];
            dn[c] = pd[c];
        }
    };

    // One sub-iteration over the lane's rows, top to bottom, in place: prev
    // keeps the old row above.  FIRST: bq still holds f; it also accumulates
    // the residual of the incoming iterate over the owned points and scales f
    // (h^2 f / 4 when isotropic) as it goes.
    double rsq = 0.0;
    const T hh = T(g.hh);
    auto sweep = [&](auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        T prev[C];
#pragma unroll
        for (int c = 0; c < C; ++c) prev[c] = up[c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const T wl = dpp_shift<kDppRowShr1>(x[i][C - 1]);
            const T er = dpp_shift<kDppRowShl1>(x[i][0]);
            T nw[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T w = c > 0 ? x[i][c - 1] : wl;
                const T e = c < C - 1 ? x[i][c + 1] : er;
                T we = w + e;
                // the halo registers are 0 except in the first / last lane of a
                // DPP row, where the shifted value is 0: the sum stays W + E
                if (c == 0) we = we + hw[i];
                if (c == C - 1) we = we + he[i];
                const T below = i < R - 1 ? x[i + 1][c] : dn[c];
                const T sn = prev[c] + below;
                if (FIRST) {
                    if (RES && i >= rlo && i < rhi && c >= clo && c < chi) {
                        const double wa = c > 0 ? (double)w : (double)wl + (double)hw[i];
                        const double ea = c < C - 1 ? (double)e : (double)er + (double)he[i];
                        const double rr = res2((double)bq[i][c], (double)x[i][c], wa, ea,
                                               (double)prev[c], (double)below, g.wx, g.wy);
                        rsq += rr * rr;
                    }
                    if (ISO) bq[i][c] = (hh * bq[i][c]) * T(0.25);
                }
                if (ISO) nw[c] = fma_quarter(we + sn, bq[i][c]);
                else nw[c] = (bq[i][c] + (wx * we + wy * sn)) * dinv;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                prev[c] = x[i][c];
                x[i][c] = nw[c];
            }
        }
    };

    // step 2: nsub sub-iterations with the halo frozen
    exchange(0);
    sweep(std::true_type{});
    for (int it = 1; it < nsub; ++it) {
        exchange(it & 1);
        sweep(std::false_type{});
    }

    // step 3: owned points back to global memory
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (i >= rlo && i < rhi && c >= clo && c < chi) xout[base + (int64_t)i * ld + c] = x[i][c];

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
        if (read_status(red.ctrl) != ST_RUNNING) return;
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
// 1D hierarchical cycle.  Tiles of TT points; a workgroup holds G = kNT / TT
// tiles (TT <= kNT) or one tile with TT / kNT points per thread.
// ============================================================================
template <typename T, int TT, bool RES>
__global__ __launch_bounds__(kNT) void k_cycle1d(Geom1 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 int s, Red red, double tol)
{
    if (RES) {
        if (read_status(red.ctrl) != ST_RUNNING) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    constexpr int G = TT <= kNT ? kNT / TT : 1;
    constexpr int PER = TT <= kNT ? 1 : TT / kNT;
    constexpr int P = TT + 2;
    __shared__ T buf[2][G * P];

    const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t n = g.n;
    const int ni = n < TT ? (int)n : TT;  // points per tile
    const int ntile = (int)g.nt;
    const int nint = n > 0x7fffffff ? 0x7fffffff : (int)n;

    for (int i = threadIdx.x; i < G * P; i += kNT) {
        const int gi = i / P, lc = i - gi * P;
        const int64_t tile = blk * G + gi;
        T v = T(0);
        if (tile < ntile) {
            const int64_t gp = (int64_t)axis_origin(nint, TT, g.o, (int)tile) + lc - 1;
            if (gp >= 0 && gp < n) v = xin[gp];
        }
        buf[0][i] = v;
        buf[1][i] = v;
    }

    const int gi = TT <= kNT ? (int)threadIdx.x / TT : 0;
    const int64_t tile = blk * G + gi;
    const bool live = tile < ntile;
    const int64_t x0 = live ? axis_origin(nint, TT, g.o, (int)tile) : 0;
    const int lo = live ? axis_own_begin(nint, TT, g.o, (int)tile) - (int)x0 : 0;
    const int hi = live ? axis_own_end(nint, TT, g.o, (int)tile, ntile) - (int)x0 : 0;
    const T hh = T(g.hh);
    T fb[PER], val[PER];
    double fr[RES ? PER : 1];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int lc = TT <= kNT ? (int)threadIdx.x % TT : (int)threadIdx.x + j * kNT;
        T fv = T(0);
        if (live && lc < ni) fv = f[x0 + lc];
        fb[j] = hh * fv;
        if (RES) fr[RES ? j : 0] = (double)fv;
        val[j] = T(0);
    }
    __syncthreads();

    double rsq = 0.0;
    if (RES) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int lc = TT <= kNT ? (int)threadIdx.x % TT : (int)threadIdx.x + j * kNT;
            if (live && lc >= lo && lc < hi) {
                const int a = gi * P + lc + 1;
                const double rr = res1(fr[RES ? j : 0], (double)buf[0][a], (double)buf[0][a - 1],
                                       (double)buf[0][a + 1], g.w1);
                rsq += rr * rr;
            }
        }
    }

    for (int k = 0; k < s; ++k) {
        const T *cur = buf[k & 1];
        T *nxt = buf[(k & 1) ^ 1];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int lc = TT <= kNT ? (int)threadIdx.x % TT : (int)threadIdx.x + j * kNT;
            if (live && lc < ni) {
                const int a = gi * P + lc + 1;
                const T v = upd1<T>(fb[j], cur[a - 1], cur[a + 1]);
                nxt[a] = v;
                val[j] = v;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int lc = TT <= kNT ? (int)threadIdx.x % TT : (int)threadIdx.x + j * kNT;
        if (live && lc >= lo && lc < hi) xout[x0 + lc] = val[j];
    }

    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// 1D classical sweep / residual: one point per thread.
template <typename T, bool RES, bool SWEEP>
__global__ __launch_bounds__(kNT) void k_sweep1d(Geom1 g, const T *__restrict__ f,
                                                 const T *__restrict__ xin, T *__restrict__ xout,
                                                 Red red, double tol)
{
    if (SWEEP && RES) {
        if (read_status(red.ctrl) != ST_RUNNING) return;
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

__global__ void k_ctrl_init(Ctrl *ctrl)
{
    ctrl->r0sq = 0.0;
    ctrl->last_rsq = 0.0;
    ctrl->iter = 0;
    ctrl->done_cycle = -1;
    ctrl->status = ST_RUNNING;
    ctrl->pad = 0;
}

// Judge iterate c from n partials left by the previous kernel (one workgroup).
__global__ __launch_bounds__(kNT) void k_judge(const double *part, int n, Ctrl *ctrl, int64_t c,
                                               double tol)
{
    judge_partials<kNT>(part, n, ctrl, c, tol);
}

// ---------------------------------------------------------------- dispatch
// Register-resident shape for a TX x TY tile: C columns and R rows per lane,
// W wavefronts.  Up to 32 x 32 one wavefront holds the tile (R = TY / 4);
// taller tiles use 4 rows per lane (8 at TX = 32) and more wavefronts, which
// keeps the per-lane footprint small enough for three or more waves per SIMD.
template <int TX, int TY>
struct RegShape {
    static constexpr int C = TX / 16;
    static constexpr int R = (TX <= 64 && TY <= 32) ? TY / 4 : (TX == 32 ? 8 : 4);
    static constexpr int W = TY / (4 * R);
    static constexpr bool ok = (TX == 32 || TX == 64 || TX == 128) && TY >= 16 && TY <= 128 &&
                               W >= 1 && 4 * R * W == TY;
};

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
    constexpr int G = TT <= kNT ? kNT / TT : 1;
    const unsigned nb = (unsigned)((g.nt + G - 1) / G);
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
    const int64_t G = g.t <= kNT ? kNT / g.t : 1;
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

hipError_t launch_ctrl_init(Ctrl *ctrl, hipStream_t st)
{
    k_ctrl_init<<<1, 1, 0, st>>>(ctrl);
    return hipGetLastError();
}

}  // namespace hj
