// hj_vc_tile.h -- the variable-coefficient cycle body (one tile, LDS
// ping-pong) and the face weights, shared by the single-problem kernel
// (hj_vc.hip) and the batched one (hj_batch.hip).
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

// Threads per workgroup of the variable-coefficient cycle: every thread
// holds the five face coefficients of each of its points in VGPRs, so tiles
// of 1024 points and more take 512 threads (at most 8 points a thread).
template <int TX, int TY>
__host__ __device__ constexpr int vc_threads()
{
    return TX * TY >= 1024 ? 512 : kNT;
}

// One cycle of tile `tile` by a workgroup of NT = vc_threads threads (the
// three steps of Sec. 4.1: tile + halo into LDS, nsub sub-iterations with the
// halo frozen, owned points back).  Thread t owns column t % TX of the tile
// and rows t / TX + j NT / TX.  Returns this thread's share of ||r||^2 of xin
// over the owned points (RES), else 0.  Several tiles in a row need a barrier
// between them (LDS is reused).
template <int TX, int TY, bool RES>
__device__ __forceinline__ double lds_tile_vc(const GeomVC &g, int tile, const double *__restrict__ f,
                                              const double *__restrict__ xin, double *__restrict__ xout,
                                              int nsub)
{
    constexpr int NT = vc_threads<TX, TY>();
    static_assert(NT % TX == 0 && (TX * TY) % NT == 0, "tile/threads mismatch");
    constexpr int P = TX + 2, R = TY + 2, PER = TX * TY / NT, RSTEP = NT / TX;
    __shared__ double buf[2][R * P];

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

// Tile shapes of the variable-coefficient cycle.
#define HJ_VC_TILES(X) X(16, 16) X(16, 32) X(16, 64) X(32, 16) X(32, 32) X(32, 64) X(64, 16) X(64, 32) X(64, 64)

}  // namespace
}  // namespace hj
