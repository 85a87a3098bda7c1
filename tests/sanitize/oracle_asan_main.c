/* Runs the CPU oracle (oracle/hj_oracle.c, linked in) under AddressSanitizer
 * and UndefinedBehaviorSanitizer on small, ragged and overlapped problems:
 * every exported routine, with the checks that must hold whatever the input
 * (s = 1 cycles are classical sweeps; an overlap of 2s - 2 makes a cycle s
 * classical sweeps; solves report a finite residual).  Exit status 0 when
 * every check holds; the sanitizers abort on the first memory or UB error. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_axis_ntiles(int64_t n, int64_t t, int64_t o);
int64_t orc_axis_start(int64_t n, int64_t t, int64_t o, int64_t i);
void orc_axis_owned(int64_t n, int64_t t, int64_t o, int64_t i, int64_t *lo, int64_t *hi);
void orc_jacobi_1d(int64_t n, double h, const double *f, double *x, int64_t nsweeps);
void orc_jacobi_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, double *x, int64_t nsweeps);
void orc_hier_1d(int64_t n, double h, const double *f, double *x, int64_t t, int64_t o, int64_t s, int64_t ncycles);
void orc_hier_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, double *x, int64_t tx, int64_t ty,
                 int64_t ox, int64_t oy, int64_t s, int64_t ncycles);
double orc_residual_1d(int64_t n, double h, const double *f, const double *x, double *r);
double orc_residual_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, const double *x, double *r);
int64_t orc_solve_1d(int64_t n, double h, const double *f, double *x, int32_t method, int64_t t, int64_t o,
                     int64_t s, double tol, int64_t max_cycles, double *rel_out, double *r0_out);
int64_t orc_solve_2d(int64_t nx, int64_t ny, double hx, double hy, const double *f, double *x, int32_t method,
                     int64_t tx, int64_t ty, int64_t ox, int64_t oy, int64_t s, double tol, int64_t max_cycles,
                     double *rel_out, double *r0_out);
void orc_vc_apply_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a, const double *u, double *out);
double orc_vc_residual_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a, const double *f,
                          const double *u, double *r);
int64_t orc_vc_solve_2d(int64_t nx, int64_t ny, double hx, double hy, const double *a, const double *f, double *x,
                        int32_t method, int64_t tx, int64_t ty, int64_t ox, int64_t oy, int64_t s, double tol,
                        int64_t max_cycles, double *rel_out, double *r0_out);
void orc_vc_grad_a_2d(int64_t nx, int64_t ny, double hx, double hy, const double *u, const double *lam,
                      double *grad);

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static uint64_t rng = 88172645463325252ull;
static double uni(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}

static double *vec(int64_t n)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) v[i] = uni();
    return v;
}

static double *copy(const double *v, int64_t n)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(c, v, sizeof(double) * (size_t)n);
    return c;
}

static void one_d(int64_t n, int64_t t)
{
    double h = 1.0 / (double)(n + 1);
    double *f = vec(n), *x0 = vec(n);
    for (int64_t s = 1; s <= 5; ++s) {
        int64_t o = 2 * s - 2;
        if (o >= t) break;
        double *a = copy(x0, n), *b = copy(x0, n);
        orc_hier_1d(n, h, f, a, t, o, s, 3);
        orc_jacobi_1d(n, h, f, b, 3 * s);
        CHECK(memcmp(a, b, sizeof(double) * (size_t)n) == 0);
        free(a);
        free(b);
    }
    int64_t nt = orc_axis_ntiles(n, t, 2);
    for (int64_t i = 0; i < nt; ++i) {
        int64_t lo, hi;
        orc_axis_owned(n, t, 2, i, &lo, &hi);
        CHECK(lo <= hi && orc_axis_start(n, t, 2, i) <= lo);
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    CHECK(isfinite(orc_residual_1d(n, h, f, x0, r)));
    double *x = copy(x0, n), rel = 0, r0 = 0;
    orc_solve_1d(n, h, f, x, 0, t, t > 2 ? 2 : 0, 3, 1e-3, 200, &rel, &r0);
    CHECK(isfinite(rel) && isfinite(r0));
    orc_solve_1d(n, h, f, x, 1, 0, 0, 1, 1e-2, 200, &rel, &r0);
    CHECK(isfinite(rel));
    free(r);
    free(x);
    free(f);
    free(x0);
}

static void two_d(int64_t nx, int64_t ny, int64_t tx, int64_t ty)
{
    double hx = 1.0 / (double)(nx + 1), hy = 1.0 / (double)(ny + 1);
    int64_t m = nx * ny;
    double *f = vec(m), *x0 = vec(m);
    for (int64_t s = 1; s <= 4; ++s) {
        int64_t o = 2 * s - 2;
        if (o >= tx || o >= ty) break;
        double *a = copy(x0, m), *b = copy(x0, m);
        orc_hier_2d(nx, ny, hx, hy, f, a, tx, ty, o, o, s, 2);
        orc_jacobi_2d(nx, ny, hx, hy, f, b, 2 * s);
        CHECK(memcmp(a, b, sizeof(double) * (size_t)m) == 0);
        free(a);
        free(b);
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    CHECK(isfinite(orc_residual_2d(nx, ny, hx, hy, f, x0, r)));
    double *x = copy(x0, m), rel = 0, r0 = 0;
    orc_solve_2d(nx, ny, hx, hy, f, x, 0, tx, ty, 0, 0, 3, 1e-2, 300, &rel, &r0);
    CHECK(isfinite(rel));
    /* variable coefficients on the (ny + 2) x (nx + 2) node grid */
    int64_t na = (nx + 2) * (ny + 2);
    double *ac = (double *)malloc(sizeof(double) * (size_t)na);
    for (int64_t i = 0; i < na; ++i) ac[i] = 1.0 + 0.5 * (uni() + 0.5);
    double *u = copy(x0, m), *lam = vec(m), *g = (double *)malloc(sizeof(double) * (size_t)na);
    orc_vc_apply_2d(nx, ny, hx, hy, ac, u, r);
    CHECK(isfinite(orc_vc_residual_2d(nx, ny, hx, hy, ac, f, u, r)));
    orc_vc_solve_2d(nx, ny, hx, hy, ac, f, u, 0, tx, ty, 2, 2, 3, 0.0, 3, &rel, &r0);
    orc_vc_solve_2d(nx, ny, hx, hy, ac, f, u, 1, 0, 0, 0, 0, 1, 1e-2, 100, &rel, &r0);
    CHECK(isfinite(rel));
    orc_vc_grad_a_2d(nx, ny, hx, hy, u, lam, g);
    for (int64_t i = 0; i < na; ++i) CHECK(isfinite(g[i]));
    free(ac);
    free(u);
    free(lam);
    free(g);
    free(r);
    free(x);
    free(f);
    free(x0);
}

int main(void)
{
    const int64_t n1[] = {1, 2, 7, 32, 33, 100, 257};
    const int64_t t1[] = {4, 8, 32};
    for (size_t i = 0; i < sizeof n1 / sizeof n1[0]; ++i)
        for (size_t j = 0; j < sizeof t1 / sizeof t1[0]; ++j) one_d(n1[i], t1[j]);
    const int64_t shapes[][2] = {{1, 1}, {3, 5}, {17, 9}, {33, 40}, {64, 31}};
    const int64_t tiles[][2] = {{4, 4}, {8, 16}, {16, 8}};
    for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i)
        for (size_t j = 0; j < sizeof tiles / sizeof tiles[0]; ++j)
            two_d(shapes[i][0], shapes[i][1], tiles[j][0], tiles[j][1]);
    printf("oracle sanitizer run: %d failed checks\n", failures);
    return failures ? 1 : 0;
}
