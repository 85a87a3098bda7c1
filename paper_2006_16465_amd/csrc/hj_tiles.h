// hj_tiles.h -- the per-tile bodies of the hierarchical cycle (Sec. 3.3,
// Sec. 4.1), shared by the one-problem kernels and the batched persistent
// kernels: the update and residual formulas, the register-resident 2D tile
// and the 1D LDS tile group.  Device code only; include after hj_launch.h.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "hj_launch.h"

namespace hj {
namespace {

// Rows in R + 1 rotating register slots (no register moves, straight-line
// rounds of R + 1 sweeps) or updated in place (one move per point and sweep).
// Measured at 4096^2: rotation costs FP64 about 34 VGPRs and one wave per
// SIMD (64x128: 236 against 183 us per cycle) but saves FP32 about a tenth
// (89 against 98 us), where the registers are half the size.
template <typename T>
constexpr bool rotate_rows()
{
    return sizeof(T) == 4;
}

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

// Minimum wavefronts per SIMD the 2D register-tile kernels ask the compiler
// for (the second __launch_bounds__ argument).  FP64 tiles of 4 x 4 points a
// lane (64x64, 64x128) hold 124 VGPRs with a rolled sweep loop and 132 with
// the unrolled one: capped at 128 (occupancy 4) the compiler spills one
// double outside the loop, and the launch beats the rolled loop (4096^2,
// s = 16: 147-150 against 153-158 us); left at 132 VGPRs (occupancy 3) an
// s = 12 launch took over 200 us against 135.  Other shapes need more
// registers than 4 waves allow and are left to the compiler.
template <typename T, int C, int R>
constexpr int min_waves_2d()
{
    return (sizeof(T) == 8 && C == 4 && R == 4) ? 4 : 1;
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

// Shifted like dpp_shift, but lanes whose source lies outside the 16-lane
// row keep `old` (bound_ctrl off): a register that holds the frozen x-halo
// in the first (row_shr) or last (row_shl) lane of each row keeps it there
// while every other lane receives its neighbour's value.
template <int CTRL>
__device__ __forceinline__ double dpp_keep(double old, double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi =
        __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_keep(float old, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                                  false));
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

// LDS of BYTES bytes; every caller asking for the same size gets the same
// array, so a kernel that runs reg_tile_2d in two precisions (never both in
// one workgroup) can size it for the wider one and hold it once.
template <int BYTES>
__device__ __forceinline__ char *lds_pool()
{
    __shared__ __align__(16) char pool[BYTES];
    return pool;
}

// One cycle of tile `tile` (row-major tile index over g's partition) by a
// workgroup of 64 W threads.  Returns this thread's share of ||r||^2 of xin
// over the owned points (RES), else 0.  A caller that runs several tiles in a
// row must place a barrier between them (LDS is reused).  LB = 0: LDS arrays
// of this instantiation; LB > 0: the lds_pool sized for LB-byte elements.
template <typename T, int C, int R, int W, bool RES, bool ISO, bool ROT, int LB = 0>
__device__ __forceinline__ double reg_tile_2d(const Geom2 &g, int tile, const T *__restrict__ f,
                                              const T *__restrict__ xin, T *__restrict__ xout,
                                              int nsub)
{
    constexpr int TX = 16 * C, TY = 4 * R * W, NG = 4 * W;
    T(*s_top)[NG][TX];  // first row of each row group, by sweep parity
    T(*s_bot)[NG][TX];  // last row of each row group
    T(*s_halo)[TX];     // frozen rows -1 and TY
    if constexpr (LB == 0) {
        __shared__ T a_top[2][NG][TX];
        __shared__ T a_bot[2][NG][TX];
        __shared__ T a_halo[2][TX];
        s_top = a_top;
        s_bot = a_bot;
        s_halo = a_halo;
    } else {
        static_assert(LB >= (int)sizeof(T), "LDS pool sized for narrower elements");
        char *pool = lds_pool<(4 * NG * TX + 2 * TX) * LB>();
        s_top = reinterpret_cast<T(*)[NG][TX]>(pool);
        s_bot = reinterpret_cast<T(*)[NG][TX]>(pool + 2 * NG * TX * sizeof(T));
        s_halo = reinterpret_cast<T(*)[TX]>(pool + 4 * NG * TX * sizeof(T));
    }

    const int k = (int)threadIdx.x >> 4, j = (int)threadIdx.x & 15;
    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int64_t ld = g.ld;
    const int lr0 = k * R, lc0 = j * C;
    const int64_t base = (int64_t)(r0 + lr0) * ld + c0 + lc0;
    // LDS slot of the lane's column c in an interface row: columns go in
    // 16-byte chunks, chunk q of all 16 lanes side by side, so each 16-byte
    // LDS access of a row group covers 256 contiguous bytes (lane-strided
    // chunks left half the banks idle on every access)
    constexpr int E = 16 / (int)sizeof(T);
    auto lcol = [j](int c) {
        if constexpr (C >= E && C % E == 0) return ((c / E) * 16 + j) * E + c % E;
        else return j * C + c;
    };

    // step 1: tile, halo and f into registers / LDS (phase 0: row i in slot i).
    // The loads issue at raised wave priority, the sweeps at the base one:
    // the workgroup that is loading gets its memory instructions out ahead
    // of the sweeping workgroup's VALU work on the same SIMDs, so the two
    // phases overlap better (4 % per 4096^2 cycle, measured A/B).
    __builtin_amdgcn_s_setprio(3);
    constexpr int NS = ROT ? R + 1 : R;
    T x[NS][C], bq[R][C], hw[R], he[R];
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
            s_halo[0][lcol(c)] = r0 > 0 ? xin[(int64_t)(r0 - 1) * ld + c0 + lc0 + c] : T(0);
    }
    if (k == NG - 1) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_halo[1][lcol(c)] =
                r0 + TY < g.ny ? xin[(int64_t)(r0 + TY) * ld + c0 + lc0 + c] : T(0);
    }
    __builtin_amdgcn_s_setprio(0);
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
    auto exchange = [&]<int P>(int par) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s_top[par][k][lcol(c)] = x[P % NS][c];
            s_bot[par][k][lcol(c)] = x[(R - 1 + P) % NS][c];
        }
        __syncthreads();
        const T *pu = k == 0 ? s_halo[0] : s_bot[par][k - 1];
        const T *pd = k == NG - 1 ? s_halo[1] : s_top[par][k + 1];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            up[c] = pu[lcol(c)];
            dn[c] = pd[lcol(c)];
        }
    };

    double rsq = 0.0;
    const T hh = T(g.hh);
    if constexpr (ROT) {
    // One sub-iteration at phase P: row i of the lane sits in slot (i + P) mod NS
    // and its new value goes to the slot of row i - 1 (free once new row i is
    // formed; for row 0 the spare slot), so the sweep leaves phase P - 1 and
    // moves no registers.  FIRST: bq still holds f; it also accumulates the
    // residual of the incoming iterate over the owned points and scales f
    // (h^2 f / 4 when isotropic) as it goes.
    auto sweep = [&]<int P, bool FIRST>() {
        T above[C];
#pragma unroll
        for (int c = 0; c < C; ++c) above[c] = up[c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int cur = (i + P) % NS;
            const int dst = (i + P + NS - 1) % NS;
            const T wl = dpp_shift<kDppRowShr1>(x[cur][C - 1]);
            const T er = dpp_shift<kDppRowShl1>(x[cur][0]);
            T nw[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T w = c > 0 ? x[cur][c - 1] : wl;
                const T e = c < C - 1 ? x[cur][c + 1] : er;
                T we = w + e;
                // the halo registers are 0 except in the first / last lane of a
                // DPP row, where the shifted value is 0: the sum stays W + E
                if (c == 0) we = we + hw[i];
                if (c == C - 1) we = we + he[i];
                const T below = i < R - 1 ? x[(i + 1 + P) % NS][c] : dn[c];
                const T sn = above[c] + below;
                if (FIRST) {
                    if (RES && i >= rlo && i < rhi && c >= clo && c < chi) {
                        const double wa = c > 0 ? (double)w : (double)wl + (double)hw[i];
                        const double ea = c < C - 1 ? (double)e : (double)er + (double)he[i];
                        const double rr = res2((double)bq[i][c], (double)x[cur][c], wa, ea,
                                               (double)above[c], (double)below, g.wx, g.wy);
                        rsq += rr * rr;
                    }
                    if (ISO) bq[i][c] = (hh * bq[i][c]) * T(0.25);
                }
                if (ISO) nw[c] = fma_quarter(we + sn, bq[i][c]);
                else nw[c] = (bq[i][c] + (wx * we + wy * sn)) * dinv;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                above[c] = x[cur][c];
                x[dst][c] = nw[c];
            }
        }
    };
    auto step = [&]<int P>(int it) {
        exchange.template operator()<P>(it & 1);
        sweep.template operator()<P, false>();
    };

    // step 2: nsub sub-iterations with the halo frozen.  The first runs at
    // phase 0 and leaves phase NS - 1; full rounds of NS sweeps (phases
    // NS - 1 .. 0, straight-line code) return there; each remainder sweep
    // lowers the phase by one.
    exchange.template operator()<0>(0);
    sweep.template operator()<0, true>();
    int it = 1;
    for (; it + NS <= nsub; it += NS) {
        [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
            (step.template operator()<NS - 1 - Ps>(it + Ps), ...);
        }(std::make_integer_sequence<int, NS>{});
    }
    const int rem = nsub - it;  // 0 <= rem < NS
    [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
        ((rem > Ps ? (step.template operator()<NS - 1 - Ps>(it + Ps), 0) : 0), ...);
    }(std::make_integer_sequence<int, NS - 1>{});
    const int ph = NS - 1 - rem;

    // step 3: owned points back to global memory (row i in slot (i + ph) mod NS)
    [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
        ((ph == Ps ? ([&] {
#pragma unroll
              for (int i = 0; i < R; ++i)
#pragma unroll
                  for (int c = 0; c < C; ++c)
                      if (i >= rlo && i < rhi && c >= clo && c < chi)
                          xout[base + (int64_t)i * ld + c] = x[(i + Ps) % NS][c];
          }(), 0) : 0),
         ...);
    }(std::make_integer_sequence<int, NS>{});

    } else {
    // One sub-iteration over the lane's rows, top to bottom, in place: prev
    // keeps the old row above.  FIRST: bq still holds f; it also accumulates
    // the residual of the incoming iterate over the owned points and scales f
    // (h^2 f / 4 when isotropic) as it goes.
    auto sweep = [&](auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        T prev[C];
#pragma unroll
        for (int c = 0; c < C; ++c) prev[c] = up[c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            // x-neighbours from the lanes beside; the first / last lane of
            // each DPP row keeps the frozen halo (or the boundary 0) in hw / he
            hw[i] = dpp_keep<kDppRowShr1>(hw[i], x[i][C - 1]);
            he[i] = dpp_keep<kDppRowShl1>(he[i], x[i][0]);
            T nw[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const T w = c > 0 ? x[i][c - 1] : hw[i];
                const T e = c < C - 1 ? x[i][c + 1] : he[i];
                const T we = w + e;
                const T below = i < R - 1 ? x[i + 1][c] : dn[c];
                const T sn = prev[c] + below;
                if (FIRST) {
                    if (RES && i >= rlo && i < rhi && c >= clo && c < chi) {
                        const double rr = res2((double)bq[i][c], (double)x[i][c], (double)w, (double)e,
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

    // step 2: nsub sub-iterations with the halo frozen.  Two per loop trip:
    // each exchange's LDS buffer is then a constant, and the two sweeps
    // trade the rows' registers between them, so the loop carries no address
    // arithmetic and no register moves (80 VALU instructions per sweep and
    // wavefront against 104 at 4 x 4 points a lane); it takes a few more
    // VGPRs, which the kernels cap (min_waves_2d) to keep occupancy 4.
    exchange.template operator()<0>(0);
    sweep(std::true_type{});
    int it = 1;
    for (; it + 1 < nsub; it += 2) {
        exchange.template operator()<0>(1);
        sweep(std::false_type{});
        exchange.template operator()<0>(0);
        sweep(std::false_type{});
    }
    if (it < nsub) {
        exchange.template operator()<0>(1);
        sweep(std::false_type{});
    }

    // step 3: owned points back to global memory
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (i >= rlo && i < rhi && c >= clo && c < chi) xout[base + (int64_t)i * ld + c] = x[i][c];

    }
    return rsq;
}


// ============================================================================
// 1D hierarchical cycle.  Tiles of TT points; a workgroup holds G = kNT / TT
// tiles (TT <= kNT) or one tile with TT / kNT points per thread.
// ============================================================================
// One cycle of the tile group `blk` (tiles blk*G .. blk*G + G - 1) by a
// workgroup of kNT threads.  Returns this thread's share of ||r||^2 of xin
// over the owned points (RES), else 0.  Several groups in a row need a
// barrier between them (LDS is reused).
template <typename T, int TT, bool RES>
__device__ __forceinline__ double lds_tiles_1d(const Geom1 &g, int64_t blk, const T *__restrict__ f,
                                               const T *__restrict__ xin, T *__restrict__ xout, int s)
{
    constexpr int G = TT <= kNT ? kNT / TT : 1;
    constexpr int PER = TT <= kNT ? 1 : TT / kNT;
    constexpr int P = TT + 2;
    __shared__ T buf[2][G * P];

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

    return rsq;
}


// ============================================================================
// 1D hierarchical cycle, register-resident (TT a multiple of 64).  One
// wavefront per tile of TT = 64 P points: lane L holds points [L P, L P + P)
// of the tile in VGPRs; the neighbours of a lane's first and last points come
// from the lanes beside it through DPP whole-wavefront shifts, and lanes 0 and
// 63 take the frozen halo instead.  No LDS and no barrier: the four
// wavefronts of a workgroup run four tiles on their own.  Same update and
// residual expressions as lds_tiles_1d, so the iterates are the same bit for
// bit.
// ============================================================================
constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i - 1 of the wavefront
constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i + 1 of the wavefront
constexpr int kRegTiles1d = kNT / 64;  // tiles per workgroup

// Lanes whose source falls outside the wavefront keep `old`.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double old, double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi =
        __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float old, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                                  false));
}

// One sweep from a to b: b_i = (h^2 f_i + (a_{i-1} + a_{i+1})) / 2 in the FMA
// form fma(a_{i-1} + a_{i+1}, 1/2, h^2 f_i / 2) (equal bit for bit while the
// values are normal numbers: halving is exact and commutes with rounding).
template <typename T, int P, bool MASK>
__device__ __forceinline__ void reg_sweep_1d(const T (&a)[P], T (&b)[P], const T (&fh)[P], T haloL, T haloR,
                                             int l0, int ni)
{
    const T lft = dpp_move<kDppWaveShr1>(haloL, a[P - 1]);
    const T rgt = dpp_move<kDppWaveShl1>(haloR, a[0]);
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const T w = i > 0 ? a[i - 1] : lft;
        const T e = i + 1 < P ? a[i + 1] : rgt;
        T v = __builtin_fma(w + e, T(0.5), fh[i]);
        if (MASK) v = l0 + i < ni ? v : T(0);
        b[i] = v;
    }
}

// The cycle of one tile by its wavefront: load, residual of the incoming
// iterate over the owned points (RES), s sweeps ping-ponging two register
// arrays, write-back.  MASK: the grid is shorter than the tile (ni < TT
// points); points at or past ni read and stay 0.
template <typename T, int P, bool RES, bool MASK>
__device__ __forceinline__ double reg_tile_1d(const Geom1 &g, const T *__restrict__ fp, const T *__restrict__ xp,
                                              T *__restrict__ op, T haloL, T haloR, int l0, int ni, int lo,
                                              int hi, int s)
{
    const T hh = T(g.hh);
    T xa[P], xb[P], fh[P];
    double rsq = 0.0;
    {
        T fv[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const bool in = !MASK || l0 + i < ni;
            xa[i] = in ? xp[i] : T(0);
            fv[i] = in ? fp[i] : T(0);
        }
        if (RES) {
            const T lft = dpp_move<kDppWaveShr1>(haloL, xa[P - 1]);
            const T rgt = dpp_move<kDppWaveShl1>(haloR, xa[0]);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int lc = l0 + i;
                if (lc >= lo && lc < hi) {
                    const double w = i > 0 ? (double)xa[i - 1] : (double)lft;
                    const double e = i + 1 < P ? (double)xa[i + 1] : (double)rgt;
                    const double rr = res1((double)fv[i], (double)xa[i], w, e, g.w1);
                    rsq += rr * rr;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i) fh[i] = (hh * fv[i]) * T(0.5);
    }
    int k = 0;
    for (; k + 1 < s; k += 2) {
        reg_sweep_1d<T, P, MASK>(xa, xb, fh, haloL, haloR, l0, ni);
        reg_sweep_1d<T, P, MASK>(xb, xa, fh, haloL, haloR, l0, ni);
    }
    if (k < s) {
        reg_sweep_1d<T, P, MASK>(xa, xb, fh, haloL, haloR, l0, ni);
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int lc = l0 + i;
            if (lc >= lo && lc < hi) op[i] = xb[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            const int lc = l0 + i;
            if (lc >= lo && lc < hi) op[i] = xa[i];
        }
    }
    return rsq;
}

// One cycle of the tiles of workgroup `blk` (tiles blk*4 .. blk*4 + 3, one
// per wavefront).  Returns this thread's share of ||r||^2 of xin over the
// owned points (RES), else 0.
template <typename T, int TT, bool RES>
__device__ __forceinline__ double reg_tiles_1d(const Geom1 &g, int64_t blk, const T *__restrict__ f,
                                               const T *__restrict__ xin, T *__restrict__ xout, int s)
{
    constexpr int P = TT / 64;
    static_assert(TT % 64 == 0 && P >= 1, "register 1D tiles hold 64 P points");
    const int lane = (int)threadIdx.x & 63;
    const int64_t tile = blk * kRegTiles1d + ((int)threadIdx.x >> 6);
    const int ntile = (int)g.nt;
    if (tile >= ntile) return 0.0;

    const int64_t n = g.n;
    const int nint = n > 0x7fffffff ? 0x7fffffff : (int)n;
    const int ni = n < TT ? (int)n : TT;  // points per tile
    const int64_t x0 = axis_origin(nint, TT, g.o, (int)tile);
    const int lo = axis_own_begin(nint, TT, g.o, (int)tile) - (int)x0;
    const int hi = axis_own_end(nint, TT, g.o, (int)tile, ntile) - (int)x0;
    const int l0 = lane * P;
    const T haloL = x0 > 0 ? xin[x0 - 1] : T(0);
    const T haloR = x0 + TT < n ? xin[x0 + TT] : T(0);
    const int64_t a = x0 + l0;
    if (ni == TT) return reg_tile_1d<T, P, RES, false>(g, f + a, xin + a, xout + a, haloL, haloR, l0, ni, lo, hi, s);
    return reg_tile_1d<T, P, RES, true>(g, f + a, xin + a, xout + a, haloL, haloR, l0, ni, lo, hi, s);
}


// Tiles per workgroup of the 1D cycle, and its body: register-resident for
// tiles of 64 points and more, LDS below.
__host__ __device__ constexpr int tiles_per_block_1d(int tt)
{
    return tt % 64 == 0 ? kRegTiles1d : (tt <= kNT ? kNT / tt : 1);
}

template <typename T, int TT, bool RES>
__device__ __forceinline__ double tiles_1d(const Geom1 &g, int64_t blk, const T *__restrict__ f,
                                           const T *__restrict__ xin, T *__restrict__ xout, int s)
{
    if constexpr (TT % 64 == 0) return reg_tiles_1d<T, TT, RES>(g, blk, f, xin, xout, s);
    else return lds_tiles_1d<T, TT, RES>(g, blk, f, xin, xout, s);
}


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

}  // namespace
}  // namespace hj
