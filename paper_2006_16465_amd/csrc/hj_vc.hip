// hj_vc.hip -- variable-coefficient diffusion -div(a grad u) = f on the 2D
// grid: the hierarchical cycle, the residual, and the gradient of a loss with
// respect to the node coefficients a (adjoint face products).
//
// The operator, its face weights and the cycle body live in hj_vc_tile.h.
#include <hip/hip_runtime.h>

#include "hj_launch.h"
#include "hj_vc_tile.h"

namespace hj {
namespace {

template <int TX, int TY, bool RES>
__global__ __launch_bounds__((vc_threads<TX, TY>())) void k_cycle2d_vc(GeomVC g, const double *__restrict__ f,
                                                                    const double *__restrict__ xin,
                                                                    double *__restrict__ xout, int nsub,
                                                                    Red red, double tol)
{
    constexpr int NT = vc_threads<TX, TY>();
    if (RES) {
        if (stopped(red.ctrl, red.c)) return;
        if (blockIdx.x == 0 && red.nb_prev > 0)
            judge_partials<NT>(red.part_prev, red.nb_prev, red.ctrl, red.c - 1, tol);
    }
    const double rsq = tile_vc<TX, TY, RES>(g, xcd_tile(blockIdx.x, gridDim.x), f, xin, xout, nsub);
    if (RES) post_partial<NT>(rsq, red.part_cur);
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
    constexpr int NT = vc_threads<TX, TY>();
    if (res) k_cycle2d_vc<TX, TY, true><<<nb, NT, 0, st>>>(g, f, xin, xout, s, red, tol);
    else k_cycle2d_vc<TX, TY, false><<<nb, NT, 0, st>>>(g, f, xin, xout, s, red, tol);
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
    HJ_VC_TILES(HJ_TILE)
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
