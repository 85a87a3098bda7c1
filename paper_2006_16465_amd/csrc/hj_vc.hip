// hj_vc.hip -- variable-coefficient diffusion -div(a grad u) = f on the 2D
// grid: the hierarchical cycle, the residual, and the gradient of a loss with
// respect to the node coefficients a (adjoint face products).
//
// a holds node values on the (ny+2) x (nx+2) grid including the boundary
// nodes (leading dimension lda).  Face weights are arithmetic means of the two
// nodes they join, scaled by 1/h^2 in the face direction; the Jacobi update is
// the elemental one of Sec. 2.1 for the pentadiagonal matrix of Sec. 4 with
// per-point coefficients:
//   u <- (f + ((w u_W + e u_E) + (s u_S + n u_N))) * dinv,
//   dinv = 1 / ((w + e) + (s + n)).
// The cycle keeps the three steps of Sec. 4.1 (tile + halo into LDS, s
// sub-iterations with the halo frozen, owned points back), and overlap.
#include <hip/hip_runtime.h>

#include "hj_launch.h"

namespace hj {
namespace {

constexpr int kNT = 256;

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

template <int TX, int TY, bool RES>
__global__ __launch_bounds__(kNT) void k_cycle2d_vc(GeomVC g, const double *__restrict__ f,
                                                    const double *__restrict__ xin,
                                                    double *__restrict__ xout, int nsub, Red red,
                                                    double tol)
{
    static_assert(kNT % TX == 0 && (TX * TY) % kNT == 0, "tile/threads mismatch");
    if (RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    constexpr int P = TX + 2, R = TY + 2, PER = TX * TY / kNT, RSTEP = kNT / TX;
    __shared__ double buf[2][R * P];

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int bi = tile / g.ntx, bj = tile - bi * g.ntx;
    const int r0 = axis_origin(g.ny, TY, g.oy, bi);
    const int c0 = axis_origin(g.nx, TX, g.ox, bj);
    const int ey = g.ny < TY ? g.ny : TY;
    const int ex = g.nx < TX ? g.nx : TX;
    const int64_t ld = g.ld;

    for (int i = threadIdx.x; i < R * P; i += kNT) {
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
    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// classical sweep (SWEEP) and / or residual (RES; with r_out when !SWEEP)
template <bool RES, bool SWEEP>
__global__ __launch_bounds__(kNT) void k_sweep2d_vc(GeomVC g, const double *__restrict__ f,
                                                    const double *__restrict__ xin,
                                                    double *__restrict__ xout, Red red, double tol)
{
    if (SWEEP && RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<kNT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const int64_t total = (int64_t)g.nx * g.ny;
    const int64_t i = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * kNT + threadIdx.x;
    double rsq = 0.0;
    if (i < total) {
        const int r = (int)(i / g.nx), q = (int)(i - (int64_t)r * g.nx);
        const int64_t a = (int64_t)r * g.ld + q;
        const Face k = face_at(g, r, q);
        const double c = xin[a];
        const double uw = q > 0 ? xin[a - 1] : 0.0;
        const double ue = q + 1 < g.nx ? xin[a + 1] : 0.0;
        const double us = r > 0 ? xin[a - g.ld] : 0.0;
        const double un = r + 1 < g.ny ? xin[a + g.ld] : 0.0;
        if (SWEEP) xout[a] = (f[a] + ((k.w * uw + k.e * ue) + (k.s * us + k.n * un))) * k.dinv;
        if (RES) {
            const double rr = f[a] - ((k.w * (c - uw) + k.e * (c - ue)) + (k.s * (c - us) + k.n * (c - un)));
            if (!SWEEP && xout) xout[a] = rr;
            rsq += rr * rr;
        }
    }
    if (RES) post_partial<kNT>(rsq, red.part_cur);
}

// dL/da at every node of the (ny+2) x (nx+2) grid, summed over nb right-hand
// sides: each face between nodes P and Q contributes
// -(1/2) (u_P - u_Q)(lam_P - lam_Q) / h^2 to both nodes (u = lam = 0 on the
// boundary).  Gathered per node, no atomics.
__global__ __launch_bounds__(kNT) void k_grad_a_vc(GeomVC g, const double *__restrict__ u,
                                                   const double *__restrict__ lam, int nb,
                                                   int64_t bstride, double *__restrict__ grad,
                                                   int64_t ldg)
{
    const int64_t total = (int64_t)(g.nx + 2) * (g.ny + 2);
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i >= total) return;
    const int R = (int)(i / (g.nx + 2)), Q = (int)(i - (int64_t)R * (g.nx + 2));
    const int r = R - 1, q = Q - 1;  // interior coordinates of the node
    auto in = [&](int rr, int qq) { return rr >= 0 && rr < g.ny && qq >= 0 && qq < g.nx; };
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double *ub = u + (int64_t)b * bstride;
        const double *lb = lam + (int64_t)b * bstride;
        auto U = [&](int rr, int qq) { return in(rr, qq) ? ub[(int64_t)rr * g.ld + qq] : 0.0; };
        auto L = [&](int rr, int qq) { return in(rr, qq) ? lb[(int64_t)rr * g.ld + qq] : 0.0; };
        const double u0 = U(r, q), l0 = L(r, q);
        double t = 0.0;
        if (r >= 0 && r < g.ny) {  // x faces exist in interior rows
            if (q - 1 >= -1) t += (u0 - U(r, q - 1)) * (l0 - L(r, q - 1)) * g.ihx2;
            if (q + 1 <= g.nx) t += (u0 - U(r, q + 1)) * (l0 - L(r, q + 1)) * g.ihx2;
        }
        if (q >= 0 && q < g.nx) {  // y faces exist in interior columns
            if (r - 1 >= -1) t += (u0 - U(r - 1, q)) * (l0 - L(r - 1, q)) * g.ihy2;
            if (r + 1 <= g.ny) t += (u0 - U(r + 1, q)) * (l0 - L(r + 1, q)) * g.ihy2;
        }
        acc += -0.5 * t;
    }
    grad[(int64_t)R * ldg + Q] = acc;
}

template <int TX, int TY>
hipError_t cyc_vc(const GeomVC &g, int s, bool res, const double *f, const double *xin, double *xout,
                  const Red &red, double tol, hipStream_t st)
{
    const unsigned nb = (unsigned)((int64_t)g.ntx * g.nty);
    if (res) k_cycle2d_vc<TX, TY, true><<<nb, kNT, 0, st>>>(g, f, xin, xout, s, red, tol);
    else k_cycle2d_vc<TX, TY, false><<<nb, kNT, 0, st>>>(g, f, xin, xout, s, red, tol);
    return hipGetLastError();
}

}  // namespace

int64_t cycle_vc_blocks(const GeomVC &g) { return (int64_t)g.ntx * g.nty; }
int64_t sweep_vc_blocks(const GeomVC &g) { return ((int64_t)g.nx * g.ny + kNT - 1) / kNT; }

hipError_t launch_cycle_vc(const GeomVC &g, int s, bool res, const double *f, const double *xin,
                           double *xout, const Red &red, double tol, hipStream_t st)
{
#define HJ_TILE(a, b) \
    if (g.tx == a && g.ty == b) return cyc_vc<a, b>(g, s, res, f, xin, xout, red, tol, st);
    HJ_TILE(16, 16) HJ_TILE(16, 32) HJ_TILE(16, 64)
    HJ_TILE(32, 16) HJ_TILE(32, 32) HJ_TILE(32, 64)
    HJ_TILE(64, 16) HJ_TILE(64, 32) HJ_TILE(64, 64)
#undef HJ_TILE
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_vc(const GeomVC &g, bool res, const double *f, const double *xin, double *xout,
                           const Red &red, double tol, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep_vc_blocks(g);
    if (res) k_sweep2d_vc<true, true><<<nb, kNT, 0, st>>>(g, f, xin, xout, red, tol);
    else k_sweep2d_vc<false, true><<<nb, kNT, 0, st>>>(g, f, xin, xout, red, tol);
    return hipGetLastError();
}

hipError_t launch_resid_vc(const GeomVC &g, const double *f, const double *x, double *r_out,
                           double *part, hipStream_t st)
{
    const unsigned nb = (unsigned)sweep_vc_blocks(g);
    const Red red{part, nullptr, nullptr, 0, 0};
    k_sweep2d_vc<true, false><<<nb, kNT, 0, st>>>(g, f, x, r_out, red, -1.0);
    return hipGetLastError();
}

hipError_t launch_grad_a_vc(const GeomVC &g, const double *u, const double *lam, int nb,
                            int64_t bstride, double *grad, int64_t ldg, hipStream_t st)
{
    const int64_t total = (int64_t)(g.nx + 2) * (g.ny + 2);
    k_grad_a_vc<<<(unsigned)((total + kNT - 1) / kNT), kNT, 0, st>>>(g, u, lam, nb, bstride, grad, ldg);
    return hipGetLastError();
}

}  // namespace hj
