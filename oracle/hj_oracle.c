/*
 * hj_oracle.c -- CPU FP64 oracle for hierarchical Jacobi on the 1D 3-point and
 * 2D 5-point Poisson systems with homogeneous Dirichlet boundaries.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * statement of what the GPU path must compute.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * library never links, loads or calls it, and it shares no code, header or
 * constant with the HIP sources.
 *
 * Paper: Islam & Wang, "Hierarchical Jacobi Iteration for Structured Matrices
 * on GPUs using Shared Memory" (arXiv:2006.16465).
 *
 *   classical Jacobi   : Sec. 2.1 eq. (jacobi-elemental); Sec. 3.1 (two
 *                        containers, sweep, swap); 1D Poisson update Sec. 3.4
 *                        eq. (jacobi-stencil-1d-poisson); 2D update Sec. 4.2.
 *   hierarchical cycle : Sec. 3.3 (three steps: copy subdomain plus one-cell
 *                        halo, k sub-iterations with the halo untouched, copy
 *                        the interior back); 2D version Sec. 4.1.
 *   overlap            : Sec. 3.5 (even overlap, left/right halves) and
 *                        Sec. 4.3 (2D: the subdomain where the point is farther
 *                        from the edge in x and in y supplies the value).
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - global double buffer: every tile of a cycle reads the previous global
 *     iterate; the halo stays frozen at that iterate for all s sweeps, in both
 *     local containers (Sec. 3.3; Appendix A loads the halo into both).
 *   - the result is taken from container s mod 2 (odd s allowed).
 *   - 2D diagonal is 2/hx^2 + 2/hy^2 (the printed d in Sec. 4.2 is garbled;
 *     the update formula printed beside it fixes this value).
 *   - update association, with h^2 f rounded once:
 *       1D:        (h^2 f + (W + E)) * 0.5
 *       2D hx==hy: (h^2 f + ((W + E) + (S + N))) * 0.25
 *       2D else:   (f + (wx (W + E) + wy (S + N))) * dinv,
 *                  wx = 1/hx^2, wy = 1/hy^2, dinv = 1/(2 wx + 2 wy).
 *     Compiled with -ffp-contract=off so no multiply-add is fused.
 *   - tiles along an axis of n points with tile t and overlap o: if n <= t one
 *     tile covers [0, n); otherwise ceil((n - o) / (t - o)) full tiles at
 *     stride t - o (the paper's operational-block count, Sec. 3.5), the last
 *     one moved left to end at n.  Where two neighbouring tiles overlap in
 *     [a, b), the left tile writes the first ceil((b - a) / 2) points and the
 *     right tile the rest (each point goes to the tile where it is farther
 *     from the frozen edge; an exact tie goes left).
 *   - residual r = f - A x over interior points; norms are 2-norms summed with
 *     Neumaier compensation; convergence when ||r_n|| <= tol * ||r_0||.
 *
 * An FP32 section (orc_*_f32) carries the same sweeps and cycles out in single
 * precision for checking an FP32 instantiation; its readings are stated there.
 *
 * Layout: 1D arrays hold the n interior points; 2D arrays are row-major
 * [ny][nx] (row = y index, column = x index), interior points only.  Points
 * outside the domain read as the Dirichlet value 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>

/* Loops over fewer point updates than this run on one thread: a parallel
 * region costs more than such a loop (and far more when several processes
 * share the cores).  Each point is computed on its own, so the thread count
 * never changes a result. */
#define PAR_MIN_POINTS ((int64_t)1 << 16)
#endif

/* ------------------------------------------------------------------ */
/* Axis partition into tiles (Sec. 3.3 subdomains, Sec. 3.5 overlap)   */
/* ------------------------------------------------------------------ */

int64_t orc_axis_ntiles(int64_t n, int64_t t, int64_t o)
{
    if (n <= t) return 1;
    int64_t stride = t - o;
    return (n - o + stride - 1) / stride;
}

int64_t orc_axis_start(int64_t n, int64_t t, int64_t o, int64_t i)
{
    if (n <= t) return 0;
    int64_t st = i * (t - o);
    if (st + t > n) st = n - t;
    return st;
}

static int64_t axis_extent(int64_t n, int64_t t) { return n < t ? n : t; }

/* owned window [*lo, *hi) of tile i */
void orc_axis_owned(int64_t n, int64_t t, int64_t o, int64_t i, int64_t *lo, int64_t *hi)
{
    int64_t nt = orc_axis_ntiles(n, t, o);
    int64_t ext = axis_extent(n, t);
    if (i == 0) {
        *lo = 0;
    } else {
        int64_t a = orc_axis_start(n, t, o, i);
        int64_t b = orc_axis_start(n, t, o, i - 1) + ext;
        *lo = a + (b - a + 1) / 2;
    }
    if (i == nt - 1) {
        *hi = n;
    } else {
        int64_t a = orc_axis_start(n, t, o, i + 1);
        int64_t b = orc_axis_start(n, t, o, i) + ext;
        *hi = a + (b - a + 1) / 2;
    }
}

/* ------------------------------------------------------------------ */
/* Point updates (Sec. 3.4 and Sec. 4.2 update equations)              */
/* ------------------------------------------------------------------ */

static double upd1(double bh, double w, double e)
{
    return (bh + (w + e)) * 0.5;
}

typedef struct {
    int iso;          /* hx == hy */
    double hh;        /* h*h when iso */
    double wx, wy, dinv;
} coef2;

static coef2 make_coef2(double hx, double hy)
{
    coef2 c;
    c.iso = (hx == hy);
    c.hh = hx * hx;
    c.wx = 1.0 / (hx * hx);
    c.wy = 1.0 / (hy * hy);
    c.dinv = 1.0 / (2.0 * c.wx + 2.0 * c.wy);
    return c;
}

static double upd2(const coef2 *c, double f, double w, double e, double s, double n)
{
    if (c->iso) {
        double bh = c->hh * f;
        return (bh + ((w + e) + (s + n))) * 0.25;
    }
    return (f + (c->wx * (w + e) + c->wy * (s + n))) * c->dinv;
}

/* ------------------------------------------------------------------ */
/* Classical Jacobi (Sec. 3.1): two containers, sweep, swap             */
/* ------------------------------------------------------------------ */

/* one classical sweep cur -> nxt (distinct arrays) */
static void jacobi_sweep_1d(int64_t n, double h, const double *f, const double *cur, double *nxt)
{
    double hh = h * h;
    for (int64_t i = 0; i < n; ++i) {
        double w = i > 0 ? cur[i - 1] : 0.0;
        double e = i < n - 1 ? cur[i + 1] : 0.0;
        nxt[i] = upd1(hh * f[i], w, e);
    }
}

void orc_jacobi_1d(int64_t n, double h, const double *f, double *x, int64_t nsweeps)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *cur = x, *nxt = y;
    for (int64_t k = 0; k < nsweeps; ++k) {
        jacobi_sweep_1d(n, h, f, cur, nxt);
        double *t = cur; cur = nxt; nxt = t;
    }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)n);
    free(y);
}

static void jacobi_sweep_2d(int64_t nx, int64_t ny, const coef2 *c, const double *f,
                            const double *cur, double *nxt)
{
    #pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN_POINTS)
    for (int64_t r = 0; r < ny; ++r) {
        for (int64_t q = 0; q < nx; ++q) {
            double w = q > 0 ? cur[r * nx + q - 1] : 0.0;
            double e = q < nx - 1 ? cur[r * nx + q + 1] : 0.0;
            double s = r > 0 ? cur[(r - 1) * nx + q] : 0.0;
            double nn = r < ny - 1 ? cur[(r + 1) * nx + q] : 0.0;
            nxt[r * nx + q] = upd2(c, f[r * nx + q], w, e, s, nn);
        }
    }
}

void orc_jacobi_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f,
                   double *x, int64_t nsweeps)
{
    coef2 c = make_coef2(hx, hy);
    double *y = (double *)malloc(sizeof(double) * (size_t)(nx * ny));
    double *cur = x, *nxt = y;
    for (int64_t k = 0; k < nsweeps; ++k) {
        jacobi_sweep_2d(nx, ny, &c, f, cur, nxt);
        double *t = cur; cur = nxt; nxt = t;
    }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)(nx * ny));
    free(y);
}

/* ------------------------------------------------------------------ */
/* Hierarchical cycle (Sec. 3.3 steps 1-3; overlap Sec. 3.5)            */
/* ------------------------------------------------------------------ */

/* one cycle: xin -> xout (distinct arrays) */
static void hier_cycle_1d(int64_t n, double h, const double *f, const double *xin,
                          double *xout, int64_t t, int64_t o, int64_t s)
{
    double hh = h * h;
    int64_t nt = orc_axis_ntiles(n, t, o);
    int64_t ext = axis_extent(n, t);
    #pragma omp parallel for schedule(static) if (nt * ext * s >= PAR_MIN_POINTS)
    for (int64_t ti = 0; ti < nt; ++ti) {
        int64_t x0 = orc_axis_start(n, t, o, ti);
        /* step 1: copy the subdomain plus one point each side into both
         * containers; outside the domain is the Dirichlet value 0 */
        double *L[2];
        L[0] = (double *)malloc(sizeof(double) * (size_t)(ext + 2));
        L[1] = (double *)malloc(sizeof(double) * (size_t)(ext + 2));
        for (int64_t j = -1; j <= ext; ++j) {
            int64_t g = x0 + j;
            double v = (g >= 0 && g < n) ? xin[g] : 0.0;
            L[0][j + 1] = v;
            L[1][j + 1] = v;
        }
        /* step 2: s sub-iterations on the interior, halo untouched */
        for (int64_t k = 0; k < s; ++k) {
            const double *src = L[k % 2];
            double *dst = L[(k + 1) % 2];
            for (int64_t j = 0; j < ext; ++j)
                dst[j + 1] = upd1(hh * f[x0 + j], src[j], src[j + 2]);
        }
        /* step 3: the owned part of the interior goes back to global memory */
        const double *res = L[s % 2];
        int64_t lo, hi;
        orc_axis_owned(n, t, o, ti, &lo, &hi);
        for (int64_t g = lo; g < hi; ++g) xout[g] = res[g - x0 + 1];
        free(L[0]);
        free(L[1]);
    }
}

static void hier_cycle_2d(int64_t nx, int64_t ny, const coef2 *c, const double *f,
                          const double *xin, double *xout, int64_t tx, int64_t ty,
                          int64_t ox, int64_t oy, int64_t s)
{
    int64_t ntx = orc_axis_ntiles(nx, tx, ox), nty = orc_axis_ntiles(ny, ty, oy);
    int64_t ex = axis_extent(nx, tx), ey = axis_extent(ny, ty);
    int64_t p = ex + 2; /* local pitch */
    #pragma omp parallel for schedule(static) if (ntx * nty * ex * ey * s >= PAR_MIN_POINTS)
    for (int64_t tid = 0; tid < ntx * nty; ++tid) {
        int64_t bi = tid / ntx, bj = tid % ntx;
        int64_t r0 = orc_axis_start(ny, ty, oy, bi);
        int64_t c0 = orc_axis_start(nx, tx, ox, bj);
        double *L[2];
        L[0] = (double *)malloc(sizeof(double) * (size_t)(p * (ey + 2)));
        L[1] = (double *)malloc(sizeof(double) * (size_t)(p * (ey + 2)));
        /* step 1: subdomain plus one-point halo into both containers */
        for (int64_t r = -1; r <= ey; ++r) {
            for (int64_t q = -1; q <= ex; ++q) {
                int64_t gr = r0 + r, gq = c0 + q;
                double v = (gr >= 0 && gr < ny && gq >= 0 && gq < nx) ? xin[gr * nx + gq] : 0.0;
                L[0][(r + 1) * p + (q + 1)] = v;
                L[1][(r + 1) * p + (q + 1)] = v;
            }
        }
        /* step 2: s sub-iterations, halo frozen */
        for (int64_t k = 0; k < s; ++k) {
            const double *src = L[k % 2];
            double *dst = L[(k + 1) % 2];
            for (int64_t r = 0; r < ey; ++r) {
                for (int64_t q = 0; q < ex; ++q) {
                    int64_t a = (r + 1) * p + (q + 1);
                    dst[a] = upd2(c, f[(r0 + r) * nx + (c0 + q)],
                                  src[a - 1], src[a + 1], src[a - p], src[a + p]);
                }
            }
        }
        /* step 3: owned window of the interior back to global memory */
        const double *res = L[s % 2];
        int64_t rlo, rhi, qlo, qhi;
        orc_axis_owned(ny, ty, oy, bi, &rlo, &rhi);
        orc_axis_owned(nx, tx, ox, bj, &qlo, &qhi);
        for (int64_t gr = rlo; gr < rhi; ++gr)
            for (int64_t gq = qlo; gq < qhi; ++gq)
                xout[gr * nx + gq] = res[(gr - r0 + 1) * p + (gq - c0 + 1)];
        free(L[0]);
        free(L[1]);
    }
}

void orc_hier_1d(int64_t n, double h, const double *f, double *x, int64_t t, int64_t o,
                 int64_t s, int64_t ncycles)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *cur = x, *nxt = y;
    for (int64_t c = 0; c < ncycles; ++c) {
        hier_cycle_1d(n, h, f, cur, nxt, t, o, s);
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)n);
    free(y);
}

void orc_hier_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, double *x,
                 int64_t tx, int64_t ty, int64_t ox, int64_t oy, int64_t s, int64_t ncycles)
{
    coef2 c = make_coef2(hx, hy);
    double *y = (double *)malloc(sizeof(double) * (size_t)(nx * ny));
    double *cur = x, *nxt = y;
    for (int64_t k = 0; k < ncycles; ++k) {
        hier_cycle_2d(nx, ny, &c, f, cur, nxt, tx, ty, ox, oy, s);
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)(nx * ny));
    free(y);
}

/* ------------------------------------------------------------------ */
/* FP32 sweeps and cycles                                               */
/* ------------------------------------------------------------------ */
/*
 * The paper computes in double precision (Sec. 3.4, Sec. 4.2).  These are
 * the same classical sweeps and hierarchical cycles carried out in single
 * precision, for checking an FP32 instantiation bit for bit.  Readings:
 *   - the coefficients are formed in FP64 from the spacings, exactly as
 *     above (h*h, 1/hx^2, 1/hy^2, 1/(2 wx + 2 wy)), then rounded once to FP32;
 *   - every operation of an update is an FP32 operation, in the association
 *     of the FP64 updates: h^2 f is the FP32 product of the rounded h^2 and f.
 * Kept apart from the FP64 code above so that nothing there changes.
 */

static float upd1f(float bh, float w, float e)
{
    return (bh + (w + e)) * 0.5f;
}

typedef struct {
    int iso;
    float hh, wx, wy, dinv;
} coef2f;

static coef2f make_coef2f(double hx, double hy)
{
    const double wx = 1.0 / (hx * hx), wy = 1.0 / (hy * hy);
    coef2f c;
    c.iso = (hx == hy);
    c.hh = (float)(hx * hx);
    c.wx = (float)wx;
    c.wy = (float)wy;
    c.dinv = (float)(1.0 / (2.0 * wx + 2.0 * wy));
    return c;
}

static float upd2f(const coef2f *c, float f, float w, float e, float s, float n)
{
    if (c->iso) {
        float bh = c->hh * f;
        return (bh + ((w + e) + (s + n))) * 0.25f;
    }
    return (f + (c->wx * (w + e) + c->wy * (s + n))) * c->dinv;
}

void orc_jacobi_1d_f32(int64_t n, double h, const float *f, float *x, int64_t nsweeps)
{
    const float hh = (float)(h * h);
    float *y = (float *)malloc(sizeof(float) * (size_t)n);
    float *cur = x, *nxt = y;
    for (int64_t k = 0; k < nsweeps; ++k) {
        for (int64_t i = 0; i < n; ++i) {
            float w = i > 0 ? cur[i - 1] : 0.0f;
            float e = i < n - 1 ? cur[i + 1] : 0.0f;
            nxt[i] = upd1f(hh * f[i], w, e);
        }
        float *t = cur; cur = nxt; nxt = t;
    }
    if (cur != x) memcpy(x, cur, sizeof(float) * (size_t)n);
    free(y);
}

void orc_jacobi_2d_f32(int64_t nx, int64_t ny, double hx, double hy, const float *f, float *x,
                       int64_t nsweeps)
{
    const coef2f c = make_coef2f(hx, hy);
    float *y = (float *)malloc(sizeof(float) * (size_t)(nx * ny));
    float *cur = x, *nxt = y;
    for (int64_t k = 0; k < nsweeps; ++k) {
        #pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN_POINTS)
        for (int64_t r = 0; r < ny; ++r) {
            for (int64_t q = 0; q < nx; ++q) {
                float w = q > 0 ? cur[r * nx + q - 1] : 0.0f;
                float e = q < nx - 1 ? cur[r * nx + q + 1] : 0.0f;
                float so = r > 0 ? cur[(r - 1) * nx + q] : 0.0f;
                float no = r < ny - 1 ? cur[(r + 1) * nx + q] : 0.0f;
                nxt[r * nx + q] = upd2f(&c, f[r * nx + q], w, e, so, no);
            }
        }
        float *t = cur; cur = nxt; nxt = t;
    }
    if (cur != x) memcpy(x, cur, sizeof(float) * (size_t)(nx * ny));
    free(y);
}

/* the three steps of Sec. 3.3 for one tile of a 1D cycle, in FP32 */
void orc_hier_1d_f32(int64_t n, double h, const float *f, float *x, int64_t t, int64_t o,
                     int64_t s, int64_t ncycles)
{
    const float hh = (float)(h * h);
    const int64_t nt = orc_axis_ntiles(n, t, o), ext = axis_extent(n, t);
    float *y = (float *)malloc(sizeof(float) * (size_t)n);
    float *L0 = (float *)malloc(sizeof(float) * (size_t)(ext + 2));
    float *L1 = (float *)malloc(sizeof(float) * (size_t)(ext + 2));
    float *cur = x, *nxt = y;
    for (int64_t cyc = 0; cyc < ncycles; ++cyc) {
        for (int64_t ti = 0; ti < nt; ++ti) {
            const int64_t x0 = orc_axis_start(n, t, o, ti);
            float *L[2] = {L0, L1};
            for (int64_t j = -1; j <= ext; ++j) {
                const int64_t g = x0 + j;
                const float v = (g >= 0 && g < n) ? cur[g] : 0.0f;
                L[0][j + 1] = v;
                L[1][j + 1] = v;
            }
            for (int64_t k = 0; k < s; ++k) {
                const float *src = L[k % 2];
                float *dst = L[(k + 1) % 2];
                for (int64_t j = 0; j < ext; ++j) dst[j + 1] = upd1f(hh * f[x0 + j], src[j], src[j + 2]);
            }
            const float *res = L[s % 2];
            int64_t lo, hi;
            orc_axis_owned(n, t, o, ti, &lo, &hi);
            for (int64_t g = lo; g < hi; ++g) nxt[g] = res[g - x0 + 1];
        }
        float *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != x) memcpy(x, cur, sizeof(float) * (size_t)n);
    free(L0);
    free(L1);
    free(y);
}

/* the three steps of Sec. 4.1 for every tile of a 2D cycle, in FP32 */
void orc_hier_2d_f32(int64_t nx, int64_t ny, double hx, double hy, const float *f, float *x,
                     int64_t tx, int64_t ty, int64_t ox, int64_t oy, int64_t s, int64_t ncycles)
{
    const coef2f c = make_coef2f(hx, hy);
    const int64_t ntx = orc_axis_ntiles(nx, tx, ox), nty = orc_axis_ntiles(ny, ty, oy);
    const int64_t ex = axis_extent(nx, tx), ey = axis_extent(ny, ty), p = ex + 2;
    float *y = (float *)malloc(sizeof(float) * (size_t)(nx * ny));
    float *cur = x, *nxt = y;
    for (int64_t cyc = 0; cyc < ncycles; ++cyc) {
        #pragma omp parallel for schedule(static) if (ntx * nty * ex * ey * s >= PAR_MIN_POINTS)
        for (int64_t tid = 0; tid < ntx * nty; ++tid) {
            const int64_t bi = tid / ntx, bj = tid % ntx;
            const int64_t r0 = orc_axis_start(ny, ty, oy, bi), c0 = orc_axis_start(nx, tx, ox, bj);
            float *L[2];
            L[0] = (float *)malloc(sizeof(float) * (size_t)(p * (ey + 2)));
            L[1] = (float *)malloc(sizeof(float) * (size_t)(p * (ey + 2)));
            for (int64_t r = -1; r <= ey; ++r) {
                for (int64_t q = -1; q <= ex; ++q) {
                    const int64_t gr = r0 + r, gq = c0 + q;
                    const float v = (gr >= 0 && gr < ny && gq >= 0 && gq < nx) ? cur[gr * nx + gq] : 0.0f;
                    L[0][(r + 1) * p + (q + 1)] = v;
                    L[1][(r + 1) * p + (q + 1)] = v;
                }
            }
            for (int64_t k = 0; k < s; ++k) {
                const float *src = L[k % 2];
                float *dst = L[(k + 1) % 2];
                for (int64_t r = 0; r < ey; ++r) {
                    for (int64_t q = 0; q < ex; ++q) {
                        const int64_t a = (r + 1) * p + (q + 1);
                        dst[a] = upd2f(&c, f[(r0 + r) * nx + (c0 + q)], src[a - 1], src[a + 1], src[a - p],
                                       src[a + p]);
                    }
                }
            }
            const float *res = L[s % 2];
            int64_t rlo, rhi, qlo, qhi;
            orc_axis_owned(ny, ty, oy, bi, &rlo, &rhi);
            orc_axis_owned(nx, tx, ox, bj, &qlo, &qhi);
            for (int64_t gr = rlo; gr < rhi; ++gr)
                for (int64_t gq = qlo; gq < qhi; ++gq) nxt[gr * nx + gq] = res[(gr - r0 + 1) * p + (gq - c0 + 1)];
            free(L[0]);
            free(L[1]);
        }
        float *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (cur != x) memcpy(x, cur, sizeof(float) * (size_t)(nx * ny));
    free(y);
}

/* ------------------------------------------------------------------ */
/* Residual r = f - A x and its 2-norm (Sec. 3.4 / 4.2 stopping rule)    */
/* ------------------------------------------------------------------ */

/* Neumaier-compensated sum of squares */
static double norm2_compensated(const double *r, int64_t m)
{
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double v = r[i] * r[i];
        double t = sum + v;
        if (fabs(sum) >= fabs(v)) comp += (sum - t) + v;
        else comp += (v - t) + sum;
        sum = t;
    }
    return sqrt(sum + comp);
}

/* returns ||f - A x||_2; r (length n) receives the residual when non-NULL */
double orc_residual_1d(int64_t n, double h, const double *f, const double *x, double *r)
{
    double w1 = 1.0 / (h * h);
    double *rr = r ? r : (double *)calloc((size_t)n, sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double w = i > 0 ? x[i - 1] : 0.0;
        double e = i < n - 1 ? x[i + 1] : 0.0;
        rr[i] = f[i] - w1 * ((2.0 * x[i] - w) - e);
    }
    double nrm = norm2_compensated(rr, n);
    if (!r) free(rr);
    return nrm;
}

double orc_residual_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f,
                       const double *x, double *r)
{
    double wx = 1.0 / (hx * hx), wy = 1.0 / (hy * hy);
    double *rr = r ? r : (double *)calloc((size_t)(nx * ny), sizeof(double));
    #pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN_POINTS)
    for (int64_t row = 0; row < ny; ++row) {
        for (int64_t q = 0; q < nx; ++q) {
            int64_t a = row * nx + q;
            double w = q > 0 ? x[a - 1] : 0.0;
            double e = q < nx - 1 ? x[a + 1] : 0.0;
            double s = row > 0 ? x[a - nx] : 0.0;
            double nn = row < ny - 1 ? x[a + nx] : 0.0;
            double ax = wx * ((2.0 * x[a] - w) - e) + wy * ((2.0 * x[a] - s) - nn);
            rr[a] = f[a] - ax;
        }
    }
    double nrm = norm2_compensated(rr, nx * ny);
    if (!r) free(rr);
    return nrm;
}

/* ------------------------------------------------------------------ */
/* Solve to tolerance, residual checked after every cycle               */
/* ------------------------------------------------------------------ */

/* method 0: hierarchical cycles (t, o, s); method 1: classical sweeps.
 * Returns the number of cycles (sweeps for method 1) after which the
 * relative residual first met tol, or -1 if max_cycles was reached first.
 * x holds the last iterate; *rel_out its relative residual, *r0_out the
 * initial residual norm. A zero initial residual counts as converged at 0. */
int64_t orc_solve_1d(int64_t n, double h, const double *f, double *x, int32_t method,
                     int64_t t, int64_t o, int64_t s, double tol, int64_t max_cycles,
                     double *rel_out, double *r0_out)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *cur = x, *nxt = y;
    double r0 = orc_residual_1d(n, h, f, cur, NULL);
    double rel = r0 > 0.0 ? 1.0 : 0.0;
    int64_t c = 0, done = -1;
    for (;;) {
        if (rel <= tol) { done = c; break; }
        if (c == max_cycles) break;
        if (method == 1) {
            jacobi_sweep_1d(n, h, f, cur, nxt);
        } else {
            hier_cycle_1d(n, h, f, cur, nxt, t, o, s);
        }
        double *tmp = cur; cur = nxt; nxt = tmp;
        ++c;
        double rn = orc_residual_1d(n, h, f, cur, NULL);
        rel = r0 > 0.0 ? rn / r0 : 0.0;
        if (!(rel == rel) || isinf(rel)) break;
    }
    if (cur != x) memcpy(x, cur, sizeof(double) * (size_t)n);
    free(y);
    if (rel_out) *rel_out = rel;
    if (r0_out) *r0_out = r0;
    return done;
}

int64_t orc_solve_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, double *x,
                     int32_t method, int64_t tx, int64_t ty, int64_t ox, int64_t oy, int64_t s,
                     double tol, int64_t max_cycles, double *rel_out, double *r0_out)
{
    coef2 cf = make_coef2(hx, hy);
    size_t bytes = sizeof(double) * (size_t)(nx * ny);
    double *y = (double *)malloc(bytes);
    double *cur = x, *nxt = y;
    double r0 = orc_residual_2d(nx, ny, hx, hy, f, cur, NULL);
    double rel = r0 > 0.0 ? 1.0 : 0.0;
    int64_t c = 0, done = -1;
    for (;;) {
        if (rel <= tol) { done = c; break; }
        if (c == max_cycles) break;
        if (method == 1) {
            jacobi_sweep_2d(nx, ny, &cf, f, cur, nxt);
        } else {
            hier_cycle_2d(nx, ny, &cf, f, cur, nxt, tx, ty, ox, oy, s);
        }
        double *tmp = cur; cur = nxt; nxt = tmp;
        ++c;
        double rn = orc_residual_2d(nx, ny, hx, hy, f, cur, NULL);
        rel = r0 > 0.0 ? rn / r0 : 0.0;
        if (!(rel == rel) || isinf(rel)) break;
    }
    if (cur != x) memcpy(x, cur, bytes);
    free(y);
    if (rel_out) *rel_out = rel;
    if (r0_out) *r0_out = r0;
    return done;
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ================================================================== */
/* Variable-coefficient diffusion -div(a grad u) = f (general tridiagonal /
 * pentadiagonal Jacobi of Sec. 3 and Sec. 4 with per-point coefficients).
 *
 * a: node values on the (ny+2) x (nx+2) grid including the boundary nodes,
 * row-major with pitch nx+2; node (r, q) of the interior is a[(r+1)(nx+2)+q+1].
 * Face coefficients are arithmetic means of the two nodes they join.
 *   (A u)_rq = [aW (u - u_W) + aE (u - u_E)] / hx^2 + [aS (u - u_S) + aN (u - u_N)] / hy^2
 * with u = 0 outside the domain.  A is symmetric positive definite.
 * Jacobi update (Sec. 2.1 elemental form):
 *   u <- (f + ((aW u_W + aE u_E) / hx^2 + (aS u_S + aN u_N) / hy^2)) / dsum,
 *   dsum = (aW + aE) / hx^2 + (aS + aN) / hy^2.
 * ================================================================== */

typedef struct {
    double w, e, s, n, dinv;  /* face weights (already / h^2) and 1/diagonal */
} vc_coef;

static vc_coef vc_at(int64_t nx, double ihx2, double ihy2, const double *a, int64_t r, int64_t q)
{
    int64_t p = nx + 2;
    int64_t c = (r + 1) * p + (q + 1);
    vc_coef k;
    k.w = 0.5 * (a[c] + a[c - 1]) * ihx2;
    k.e = 0.5 * (a[c] + a[c + 1]) * ihx2;
    k.s = 0.5 * (a[c] + a[c - p]) * ihy2;
    k.n = 0.5 * (a[c] + a[c + p]) * ihy2;
    k.dinv = 1.0 / ((k.w + k.e) + (k.s + k.n));
    return k;
}

static double vc_upd(const vc_coef *k, double f, double uw, double ue, double us, double un)
{
    return (f + ((k->w * uw + k->e * ue) + (k->s * us + k->n * un))) * k->dinv;
}

/* out = A u */
void orc_vc_apply_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a, const double *u,
                     double *out)
{
    double ihx2 = 1.0 / (hx * hx), ihy2 = 1.0 / (hy * hy);
    #pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN_POINTS)
    for (int64_t r = 0; r < ny; ++r) {
        for (int64_t q = 0; q < nx; ++q) {
            vc_coef k = vc_at(nx, ihx2, ihy2, a, r, q);
            double c = u[r * nx + q];
            double uw = q > 0 ? u[r * nx + q - 1] : 0.0;
            double ue = q < nx - 1 ? u[r * nx + q + 1] : 0.0;
            double us = r > 0 ? u[(r - 1) * nx + q] : 0.0;
            double un = r < ny - 1 ? u[(r + 1) * nx + q] : 0.0;
            out[r * nx + q] = (k.w * (c - uw) + k.e * (c - ue)) + (k.s * (c - us) + k.n * (c - un));
        }
    }
}

double orc_vc_residual_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a,
                          const double *f, const double *u, double *r)
{
    double *rr = r ? r : (double *)calloc((size_t)(nx * ny), sizeof(double));
    orc_vc_apply_2d(nx, ny, hx, hy, a, u, rr);
    for (int64_t i = 0; i < nx * ny; ++i) rr[i] = f[i] - rr[i];
    double nrm = norm2_compensated(rr, nx * ny);
    if (!r) free(rr);
    return nrm;
}

static void vc_jacobi_sweep(int64_t nx, int64_t ny, double ihx2, double ihy2, const double *a,
                            const double *f, const double *cur, double *nxt)
{
    #pragma omp parallel for schedule(static) if (nx * ny >= PAR_MIN_POINTS)
    for (int64_t r = 0; r < ny; ++r) {
        for (int64_t q = 0; q < nx; ++q) {
            vc_coef k = vc_at(nx, ihx2, ihy2, a, r, q);
            double uw = q > 0 ? cur[r * nx + q - 1] : 0.0;
            double ue = q < nx - 1 ? cur[r * nx + q + 1] : 0.0;
            double us = r > 0 ? cur[(r - 1) * nx + q] : 0.0;
            double un = r < ny - 1 ? cur[(r + 1) * nx + q] : 0.0;
            nxt[r * nx + q] = vc_upd(&k, f[r * nx + q], uw, ue, us, un);
        }
    }
}

/* one hierarchical cycle for the variable-coefficient operator (Sec. 4.1 steps) */
static void vc_hier_cycle(int64_t nx, int64_t ny, double ihx2, double ihy2, const double *a,
                          const double *f, const double *xin, double *xout, int64_t tx, int64_t ty,
                          int64_t ox, int64_t oy, int64_t s)
{
    int64_t ntx = orc_axis_ntiles(nx, tx, ox), nty = orc_axis_ntiles(ny, ty, oy);
    int64_t ex = axis_extent(nx, tx), ey = axis_extent(ny, ty);
    int64_t p = ex + 2;
    #pragma omp parallel for schedule(static) if (ntx * nty * ex * ey * s >= PAR_MIN_POINTS)
    for (int64_t tid = 0; tid < ntx * nty; ++tid) {
        int64_t bi = tid / ntx, bj = tid % ntx;
        int64_t r0 = orc_axis_start(ny, ty, oy, bi);
        int64_t c0 = orc_axis_start(nx, tx, ox, bj);
        double *L[2];
        L[0] = (double *)malloc(sizeof(double) * (size_t)(p * (ey + 2)));
        L[1] = (double *)malloc(sizeof(double) * (size_t)(p * (ey + 2)));
        for (int64_t r = -1; r <= ey; ++r) {
            for (int64_t q = -1; q <= ex; ++q) {
                int64_t gr = r0 + r, gq = c0 + q;
                double v = (gr >= 0 && gr < ny && gq >= 0 && gq < nx) ? xin[gr * nx + gq] : 0.0;
                L[0][(r + 1) * p + (q + 1)] = v;
                L[1][(r + 1) * p + (q + 1)] = v;
            }
        }
        for (int64_t k = 0; k < s; ++k) {
            const double *src = L[k % 2];
            double *dst = L[(k + 1) % 2];
            for (int64_t r = 0; r < ey; ++r) {
                for (int64_t q = 0; q < ex; ++q) {
                    int64_t c = (r + 1) * p + (q + 1);
                    vc_coef kk = vc_at(nx, ihx2, ihy2, a, r0 + r, c0 + q);
                    dst[c] = vc_upd(&kk, f[(r0 + r) * nx + (c0 + q)], src[c - 1], src[c + 1],
                                    src[c - p], src[c + p]);
                }
            }
        }
        const double *res = L[s % 2];
        int64_t rlo, rhi, qlo, qhi;
        orc_axis_owned(ny, ty, oy, bi, &rlo, &rhi);
        orc_axis_owned(nx, tx, ox, bj, &qlo, &qhi);
        for (int64_t gr = rlo; gr < rhi; ++gr)
            for (int64_t gq = qlo; gq < qhi; ++gq)
                xout[gr * nx + gq] = res[(gr - r0 + 1) * p + (gq - c0 + 1)];
        free(L[0]);
        free(L[1]);
    }
}

/* method 0: hierarchical (tile, overlap, s); 1: classical.  ncycles >= 0 fixed
 * cycles when tol <= 0, else to tolerance (checked every cycle).  Returns the
 * cycle count (or -1 if max_cycles ran out), like orc_solve_2d. */
int64_t orc_vc_solve_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a,
                        const double *f, double *x, int32_t method, int64_t tx, int64_t ty,
                        int64_t ox, int64_t oy, int64_t s, double tol, int64_t max_cycles,
                        double *rel_out, double *r0_out)
{
    double ihx2 = 1.0 / (hx * hx), ihy2 = 1.0 / (hy * hy);
    size_t bytes = sizeof(double) * (size_t)(nx * ny);
    double *y = (double *)malloc(bytes);
    double *cur = x, *nxt = y;
    double r0 = orc_vc_residual_2d(nx, ny, hx, hy, a, f, cur, NULL);
    double rel = r0 > 0.0 ? 1.0 : 0.0;
    int64_t c = 0, done = -1;
    for (;;) {
        if (tol > 0.0 && rel <= tol) { done = c; break; }
        if (c == max_cycles) break;
        if (method == 1) vc_jacobi_sweep(nx, ny, ihx2, ihy2, a, f, cur, nxt);
        else vc_hier_cycle(nx, ny, ihx2, ihy2, a, f, cur, nxt, tx, ty, ox, oy, s);
        double *tmp = cur; cur = nxt; nxt = tmp;
        ++c;
        if (tol > 0.0 || c == max_cycles) {
            double rn = orc_vc_residual_2d(nx, ny, hx, hy, a, f, cur, NULL);
            rel = r0 > 0.0 ? rn / r0 : 0.0;
            if (!(rel == rel) || isinf(rel)) break;
        }
    }
    if (cur != x) memcpy(x, cur, bytes);
    free(y);
    if (rel_out) *rel_out = rel;
    if (r0_out) *r0_out = r0;
    return tol > 0.0 ? done : c;
}

/* Gradient of a loss L(u) with A(a) u = f with respect to the node values a,
 * given the forward state u and the adjoint lam (A lam = dL/du; A symmetric):
 *   dL/da = -lam^T (dA/da) u.
 * Every face between nodes P and Q carries w (u_P - u_Q)(lam_P - lam_Q) / h^2
 * (boundary nodes have u = lam = 0), with w = 1/2 for each of the two nodes in
 * the arithmetic-mean face coefficient.  grad has the layout of a. */
void orc_vc_grad_a_2d(int64_t nx, int64_t ny, double hx, double hy, const double *u,
                      const double *lam, double *grad)
{
    int64_t p = nx + 2;
    double ihx2 = 1.0 / (hx * hx), ihy2 = 1.0 / (hy * hy);
    memset(grad, 0, sizeof(double) * (size_t)(p * (ny + 2)));
    /* node value (r, q) of the extended grid; 0 on the boundary */
#define U_AT(R, Q) (((R) >= 0 && (R) < ny && (Q) >= 0 && (Q) < nx) ? u[(R) * nx + (Q)] : 0.0)
#define L_AT(R, Q) (((R) >= 0 && (R) < ny && (Q) >= 0 && (Q) < nx) ? lam[(R) * nx + (Q)] : 0.0)
    /* x faces: between (r, q) and (r, q + 1), q = -1 .. nx - 1, interior rows */
    for (int64_t r = 0; r < ny; ++r) {
        for (int64_t q = -1; q < nx; ++q) {
            double t = -(U_AT(r, q) - U_AT(r, q + 1)) * (L_AT(r, q) - L_AT(r, q + 1)) * ihx2 * 0.5;
            grad[(r + 1) * p + (q + 1)] += t;
            grad[(r + 1) * p + (q + 2)] += t;
        }
    }
    /* y faces: between (r, q) and (r + 1, q), r = -1 .. ny - 1, interior columns */
    for (int64_t r = -1; r < ny; ++r) {
        for (int64_t q = 0; q < nx; ++q) {
            double t = -(U_AT(r, q) - U_AT(r + 1, q)) * (L_AT(r, q) - L_AT(r + 1, q)) * ihy2 * 0.5;
            grad[(r + 1) * p + (q + 1)] += t;
            grad[(r + 2) * p + (q + 1)] += t;
        }
    }
#undef U_AT
#undef L_AT
}
