// hj_vc_tile.h -- the variable-coefficient cycle bodies (one tile: register
// resident, or LDS ping-pong for grids smaller than a tile) and the face
// weights, shared by the single-problem kernel (hj_vc.hip) and the batched
// one (hj_batch.hip).
//
// a holds node values on the (ny+2) x (nx+2) grid including the boundary
// nodes (leading dimension lda).  Face weights are arithmetic means of the two
// nodes they join, scaled by 1/h^2 in the face direction; the Jacobi update is
// the elemental one of Sec. 2.1 for the pentadiagonal matrix of Sec. 4 with
// per-point coefficients:
//   u <- (f + ((w u_W + e u_E) + (s u_S + n u_N))) * dinv,
//   dinv = 1 / ((w + e) + (s + n)).
#pragma once

#include <hip/hip_runtime.h>

#include "hj_tiles.h"

namespace hj {
namespace {

struct Face {
    double w, e, s, n, dinv;
};

// face weights of interior point (r, q)
__device__ __forceinline__ Face face_at(const GeomVC &g, int r, int q)
{
    const double *c = g.a + (int64_t)(r + 1) * g.lda + (q + 1);
    const double ac = c[0];
    Face k;
    k.w = 0.5 * (ac + c[-1]) * g.ihx2;
    k.e = 0.5 * (ac + c[1]) * g.ihx2;
    k.s = 0.5 * (ac + c[-g.lda]) * g.ihy2;
    k.n = 0.5 * (ac + c[g.lda]) * g.ihy2;
    k.dinv = 1.0 / ((k.w + k.e) + (k.s + k.n));
    return k;
}

// Workgroup shape of the variable-coefficient cycle on a TX x TY tile: W
// wavefronts of 16-lane row groups, each lane holding C = TX / 16 columns of
// R = 2 rows (TY = 4 R W).  Both tile bodies below run with these 64 W
// threads, so one kernel can hold both.
template <int TX, int TY>
struct VcShape {
    static constexpr int C = TX / 16, R = 2, W = TY / (4 * R), NT = 64 * W;
    static_assert(TX % 16 == 0 && TY % 8 == 0 && TX <= 64 && TY <= 64, "tile shape");
};

template <int TX, int TY>
__host__ __device__ constexpr int vc_threads()
{
    return VcShape<TX, TY>::NT;
}

// LDS bytes either body needs (one pool serves both)
template <int TX, int TY>
constexpr int vc_lds_bytes()
{
    constexpr int lds = 2 * (TX + 2) * (TY + 2) * 8;
    constexpr int reg = (4 * 4 * VcShape<TX, TY>::W * TX + 2 * TX) * 8;
    return lds > reg ? lds : reg;
}

// LDS ping-pong body, any grid (also smaller than a tile).
// One cycle of tile `tile` by a workgroup of NT = vc_threads threads (the
// three steps of Sec. 4.1: tile + halo into LDS, nsub sub-iterations with the
// halo frozen, owned points back).  Thread t owns column t % TX of the tile
// and rows t / TX + j NT / TX.  Returns this thread's share of ||r||^2 of xin
// over the owned points (RES), else 0.  Several tiles in a row need a barrier
// between them (LDS is reused).
template <int TX, int TY, bool RES>
__device__ __forceinline__ double lds_tile_vc(const GeomVC &g, int tile, const double *__restrict__ f,
                                              const double *__restrict__ xin, double *__restrict__ xout,
                                              int nsub, char *pool)
{
    constexpr int NT = vc_threads<TX, TY>();
    static_assert(NT % TX == 0 && (TX * TY) % NT == 0, "tile/threads mismatch");
    constexpr int P = TX + 2, R = TY + 2, PER = TX * TY / NT, RSTEP = NT / TX;
    double(*buf)[R * P] = reinterpret_cast<double(*)[R * P]>(pool);

    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int ey = g.ny < TY ? g.ny : TY;
    const int ex = g.nx < TX ? g.nx : TX;
    const int64_t ld = g.ld;

    for (int i = threadIdx.x; i < R * P; i += NT) {
        const int lr = i / P, lc = i - lr * P;
        const int gr = r0 + lr - 1, gc = c0 + lc - 1;
        double v = 0.0;
        if (gr >= 0 && gr < g.ny && gc >= 0 && gc < g.nx) v = xin[(int64_t)gr * ld + gc];
        buf[0][i] = v;
        buf[1][i] = v;
    }

    const int tc = threadIdx.x % TX, tr = threadIdx.x / TX;
    Face k[PER];
    double fv[PER], val[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = tr + j * RSTEP;
        const bool in = r < ey && tc < ex;
        fv[j] = in ? f[(int64_t)(r0 + r) * ld + c0 + tc] : 0.0;
        if (in) k[j] = face_at(g, r0 + r, c0 + tc);
        else k[j] = Face{0.0, 0.0, 0.0, 0.0, 0.0};
        val[j] = 0.0;
    }
    const int rlo = axis_own_begin(g.ny, TY, g.oy, bi) - r0;
    const int rhi = axis_own_end(g.ny, TY, g.oy, bi, g.nty) - r0;
    const int clo = axis_own_begin(g.nx, TX, g.ox, bj) - c0;
    const int chi = axis_own_end(g.nx, TX, g.ox, bj, g.ntx) - c0;
    const bool col_own = tc >= clo && tc < chi;
    __syncthreads();

    double rsq = 0.0;
    if (RES) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tr + j * RSTEP;
            if (col_own && r >= rlo && r < rhi) {
                const int a = (r + 1) * P + tc + 1;
                const double *b0 = buf[0];
                const double c = b0[a];
                const double ax = (k[j].w * (c - b0[a - 1]) + k[j].e * (c - b0[a + 1])) +
                                  (k[j].s * (c - b0[a - P]) + k[j].n * (c - b0[a + P]));
                const double rr = fv[j] - ax;
                rsq += rr * rr;
            }
        }
    }

    for (int it = 0; it < nsub; ++it) {
        const double *cur = buf[it & 1];
        double *nxt = buf[(it & 1) ^ 1];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int r = tr + j * RSTEP;
            if (r < ey && tc < ex) {
                const int a = (r + 1) * P + tc + 1;
                const double v = (fv[j] + ((k[j].w * cur[a - 1] + k[j].e * cur[a + 1]) +
                                           (k[j].s * cur[a - P] + k[j].n * cur[a + P]))) *
                                 k[j].dinv;
                nxt[a] = v;
                val[j] = v;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int r = tr + j * RSTEP;
        if (col_own && r >= rlo && r < rhi) xout[(int64_t)(r0 + r) * ld + c0 + tc] = val[j];
    }
    return rsq;
}

// Register-resident body for grids that hold a full tile in each direction
// (the same cycle, bit for bit).  Thread t is lane j = t % 16 of row group
// k = t / 16 and holds rows [kR, kR + R) x columns [jC, jC + C) of the tile
// with, per point, f, the east and north face weights and 1 / (sum of the
// four); a point's west face is the east face of the point to its left and
// its south face the north face of the point above (the same sums, added in
// the other order, so the same values), so only the lane's first column and
// first row keep extra ones.  x-neighbours in other lanes come from DPP row
// shifts that leave the frozen x-halo in the edge lanes; y-neighbours in
// other row groups through LDS interface rows, double-buffered by sweep
// parity (one barrier per sweep); the frozen rows -1 and TY sit in LDS.
template <int C, int R, int W, bool RES>
__device__ __forceinline__ double reg_tile_vc(const GeomVC &g, int tile, const double *__restrict__ f,
                                              const double *__restrict__ xin, double *__restrict__ xout,
                                              int nsub, char *pool)
{
    constexpr int TX = 16 * C, TY = 4 * R * W, NG = 4 * W;
    double(*s_top)[NG][TX] = reinterpret_cast<double(*)[NG][TX]>(pool);
    double(*s_bot)[NG][TX] = reinterpret_cast<double(*)[NG][TX]>(pool + 2 * NG * TX * 8);
    double(*s_halo)[TX] = reinterpret_cast<double(*)[TX]>(pool + 4 * NG * TX * 8);

    const int k = (int)threadIdx.x >> 4, j = (int)threadIdx.x & 15;
    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int64_t ld = g.ld;
    const int lr0 = k * R, lc0 = j * C;
    const int64_t base = (int64_t)(r0 + lr0) * ld + c0 + lc0;
    // 16-byte chunk q of all 16 lanes side by side in an interface row
    auto lcol = [j](int c) {
        if constexpr (C % 2 == 0) return ((c / 2) * 16 + j) * 2 + c % 2;
        else return j * C + c;
    };

    // step 1: x, f, the x-halo and the face weights into registers, the
    // frozen halo rows into LDS.  ab[ii * lda + cc] is the node of interior
    // point (r0 + lr0 + ii - 1, c0 + lc0 + cc - 1).
    double x[R][C], fv[R][C], fe[R][C], fn[R][C], di[R][C], fw0[R], fs0[C], hw[R], he[R];
    {
        const double *ab = g.a + (int64_t)(r0 + lr0) * g.lda + (c0 + lc0);
        double A[R + 2][C + 2];
#pragma unroll
        for (int ii = 0; ii < R + 2; ++ii)
#pragma unroll
            for (int cc = 0; cc < C + 2; ++cc) A[ii][cc] = ab[(int64_t)ii * g.lda + cc];
#pragma unroll
        for (int i = 0; i < R; ++i) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                x[i][c] = xin[base + (int64_t)i * ld + c];
                fv[i][c] = f[base + (int64_t)i * ld + c];
                fe[i][c] = 0.5 * (A[i + 1][c + 1] + A[i + 1][c + 2]) * g.ihx2;
                fn[i][c] = 0.5 * (A[i + 1][c + 1] + A[i + 2][c + 1]) * g.ihy2;
            }
            fw0[i] = 0.5 * (A[i + 1][1] + A[i + 1][0]) * g.ihx2;
            hw[i] = (j == 0 && c0 > 0) ? xin[base + (int64_t)i * ld - 1] : 0.0;
            he[i] = (j == 15 && c0 + TX < g.nx) ? xin[base + (int64_t)i * ld + C] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < C; ++c) fs0[c] = 0.5 * (A[1][c + 1] + A[0][c + 1]) * g.ihy2;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double w = c > 0 ? fe[i][c - 1] : fw0[i];
                const double sf = i > 0 ? fn[i - 1][c] : fs0[c];
                di[i][c] = 1.0 / ((w + fe[i][c]) + (sf + fn[i][c]));
            }
    }
    if (k == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_halo[0][lcol(c)] = r0 > 0 ? xin[(int64_t)(r0 - 1) * ld + c0 + lc0 + c] : 0.0;
    }
    if (k == NG - 1) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            s_halo[1][lcol(c)] = r0 + TY < g.ny ? xin[(int64_t)(r0 + TY) * ld + c0 + lc0 + c] : 0.0;
    }
    const int rlo = axis_own_begin(g.ny, TY, g.oy, bi) - r0 - lr0;
    const int rhi = axis_own_end(g.ny, TY, g.oy, bi, g.nty) - r0 - lr0;
    const int clo = axis_own_begin(g.nx, TX, g.ox, bj) - c0 - lc0;
    const int chi = axis_own_end(g.nx, TX, g.ox, bj, g.ntx) - c0 - lc0;

    double up[C], dn[C];
    // publish this group's first / last rows for the sweep of parity par and
    // fetch the neighbouring groups' (or the frozen halo rows); a buffer is
    // rewritten two sweeps later, after a barrier every thread reaches only
    // once its reads from it are done
    auto exchange = [&](int par) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s_top[par][k][lcol(c)] = x[0][c];
            s_bot[par][k][lcol(c)] = x[R - 1][c];
        }
        __syncthreads();
        const double *pu = k == 0 ? s_halo[0] : s_bot[par][k - 1];
        const double *pd = k == NG - 1 ? s_halo[1] : s_top[par][k + 1];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            up[c] = pu[lcol(c)];
            dn[c] = pd[lcol(c)];
        }
    };

    // step 2: one sub-iteration over the lane's rows, top to bottom, in
    // place (prev keeps the old row above).  FIRST: also the residual of the
    // incoming iterate over the owned points.
    double rsq = 0.0;
    auto sweep = [&](auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        double prev[C];
#pragma unroll
        for (int c = 0; c < C; ++c) prev[c] = up[c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            hw[i] = dpp_keep<kDppRowShr1>(hw[i], x[i][C - 1]);
            he[i] = dpp_keep<kDppRowShl1>(he[i], x[i][0]);
            double nw[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double uw = c > 0 ? x[i][c - 1] : hw[i];
                const double ue = c < C - 1 ? x[i][c + 1] : he[i];
                const double us = prev[c];
                const double un = i < R - 1 ? x[i + 1][c] : dn[c];
                const double w = c > 0 ? fe[i][c - 1] : fw0[i];
                const double sf = i > 0 ? fn[i - 1][c] : fs0[c];
                if (FIRST && RES && i >= rlo && i < rhi && c >= clo && c < chi) {
                    const double xc = x[i][c];
                    const double ax = (w * (xc - uw) + fe[i][c] * (xc - ue)) + (sf * (xc - us) + fn[i][c] * (xc - un));
                    const double rr = fv[i][c] - ax;
                    rsq += rr * rr;
                }
                nw[c] = (fv[i][c] + ((w * uw + fe[i][c] * ue) + (sf * us + fn[i][c] * un))) * di[i][c];
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                prev[c] = x[i][c];
                x[i][c] = nw[c];
            }
        }
    };
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
    return rsq;
}

// One cycle of tile `tile`: the register body when the grid holds a full
// tile in each direction (and g.reg), else the LDS body.
template <int TX, int TY, bool RES>
__device__ __forceinline__ double tile_vc(const GeomVC &g, int tile, const double *__restrict__ f,
                                          const double *__restrict__ xin, double *__restrict__ xout, int nsub)
{
    using S = VcShape<TX, TY>;
    char *pool = lds_pool<vc_lds_bytes<TX, TY>()>();
    if (g.reg && g.nx >= TX && g.ny >= TY)
        return reg_tile_vc<S::C, S::R, S::W, RES>(g, tile, f, xin, xout, nsub, pool);
    return lds_tile_vc<TX, TY, RES>(g, tile, f, xin, xout, nsub, pool);
}

// Tile shapes of the variable-coefficient cycle.
#define HJ_VC_TILES(X) X(16, 16) X(16, 32) X(16, 64) X(32, 16) X(32, 32) X(32, 64) X(64, 16) X(64, 32) X(64, 64)

}  // namespace
}  // namespace hj
