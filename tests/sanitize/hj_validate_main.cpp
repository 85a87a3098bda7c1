// Runs every validation path of libhj's C ABI (include/hj.h) under the host
// AddressSanitizer and UndefinedBehaviorSanitizer: each call carries one bad
// argument and must return its error status before touching the GPU, with a
// detail string.  No GPU is needed (pointers are never dereferenced).  Exit
// status 0 when every call returns the expected status.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hj.h"

static int failures = 0;
static void expect(hj_status got, hj_status want, int line)
{
    if (got != want || (want != HJ_OK && !hj_last_error()[0])) {
        std::fprintf(stderr, "line %d: status %d (want %d), detail '%s'\n", line, (int)got, (int)want,
                     hj_last_error());
        ++failures;
    }
}
#define EXPECT(call, want) expect((call), (want), __LINE__)

int main()
{
    void *const FAKE = reinterpret_cast<void *>(0x10000);
    void *const ODD = reinterpret_cast<void *>(0x10004);
    hj_params p;
    hj_params_default(&p);
    hj_info info;

    // 2D solves (both entry points share the checks)
    for (int e = 0; e < 2; ++e) {
        auto s2 = [&](int64_t nx, int64_t ny, int64_t ld, double hx, double hy, int dt, const void *f, void *x,
                      const hj_params *q) {
            return e == 0 ? hj_solve_2d(nx, ny, ld, hx, hy, (hj_dtype)dt, f, x, q, nullptr, &info)
                          : hj_solve_2d_noalloc(nx, ny, ld, hx, hy, (hj_dtype)dt, f, x, q, nullptr, &info);
        };
        EXPECT(s2(0, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 7, 0.1, 0.1, 0, FAKE, FAKE, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 8, -1.0, 0.1, 0, FAKE, FAKE, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 9, FAKE, FAKE, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, nullptr, FAKE, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, ODD, &p), HJ_ERR_INVALID_ARG);
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, nullptr), HJ_ERR_INVALID_ARG);
        hj_params q = p;
        q.s = 0;
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, &q), HJ_ERR_INVALID_ARG);
        q = p;
        q.overlap_x = q.tile_x;
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, &q), HJ_ERR_INVALID_ARG);
        q = p;
        q.tile_x = 48;
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, &q), HJ_ERR_UNSUPPORTED);
        q = p;
        q.flags = 64;
        EXPECT(s2(8, 8, 8, 0.1, 0.1, 0, FAKE, FAKE, &q), HJ_ERR_INVALID_ARG);
    }
    EXPECT(hj_solve_2d_noalloc(4096, 4096, 4096, 0.1, 0.1, HJ_F64, FAKE, FAKE, &p, nullptr, &info),
           HJ_ERR_INVALID_ARG);

    // 1D
    EXPECT(hj_solve_1d(0, 0.1, HJ_F64, FAKE, FAKE, &p, nullptr, &info), HJ_ERR_INVALID_ARG);
    EXPECT(hj_solve_1d(8, 0.0, HJ_F64, FAKE, FAKE, &p, nullptr, &info), HJ_ERR_INVALID_ARG);
    EXPECT(hj_solve_1d(8, 0.1, HJ_F64, FAKE, ODD, &p, nullptr, &info), HJ_ERR_INVALID_ARG);

    // residual
    double nrm = 0.0;
    EXPECT(hj_residual(3, 8, 8, 8, 0.1, 0.1, HJ_F64, FAKE, FAKE, nullptr, &nrm, nullptr), HJ_ERR_INVALID_ARG);
    EXPECT(hj_residual(2, 8, 8, 4, 0.1, 0.1, HJ_F64, FAKE, FAKE, nullptr, &nrm, nullptr), HJ_ERR_INVALID_ARG);
    EXPECT(hj_residual(2, 8, 8, 8, 0.1, 0.1, HJ_F64, FAKE, FAKE, ODD, &nrm, nullptr), HJ_ERR_INVALID_ARG);

    // refinement
    hj_refine_params rp;
    std::memset(&rp, 0, sizeof rp);
    rp.inner = p;
    rp.inner.rel_tol = 1e-4;
    rp.rel_tol = 1e-10;
    rp.max_outer = 4;
    hj_refine_info ri;
    hj_refine_params bad = rp;
    bad.max_outer = 0;
    EXPECT(hj_solve_2d_refined(8, 8, 8, 0.1, 0.1, (const double *)FAKE, (double *)FAKE, &bad, nullptr, &ri),
           HJ_ERR_INVALID_ARG);
    bad = rp;
    bad.switch_min_cycles = -3;
    EXPECT(hj_solve_2d_refined(8, 8, 8, 0.1, 0.1, (const double *)FAKE, (double *)FAKE, &bad, nullptr, &ri),
           HJ_ERR_INVALID_ARG);
    bad = rp;
    bad.switch_tol = -1.0;
    EXPECT(hj_solve_2d_refined(8, 8, 8, 0.1, 0.1, (const double *)FAKE, (double *)FAKE, &bad, nullptr, &ri),
           HJ_ERR_INVALID_ARG);

    // batches
    hj_problem pr;
    std::memset(&pr, 0, sizeof pr);
    pr.dim = 2;
    pr.nx = pr.ny = pr.ld = 64;
    pr.hx = pr.hy = 0.01;
    pr.f = FAKE;
    pr.x = FAKE;
    hj_batch_params bp;
    std::memset(&bp, 0, sizeof bp);
    hj_params_default(&bp.p2);
    hj_params_default(&bp.p1);
    bp.rel_tol = 1e-6;
    bp.max_cycles = 10;
    EXPECT(hj_solve_batched(&pr, 0, &bp, nullptr, nullptr), HJ_ERR_INVALID_ARG);
    EXPECT(hj_solve_batched(nullptr, 1, &bp, nullptr, nullptr), HJ_ERR_INVALID_ARG);
    hj_problem bad_pr = pr;
    bad_pr.dim = 3;
    EXPECT(hj_solve_batched(&bad_pr, 1, &bp, nullptr, nullptr), HJ_ERR_INVALID_ARG);
    hj_batch_params bad_bp = bp;
    bad_bp.max_cycles = 0;
    EXPECT(hj_solve_batched(&pr, 1, &bad_bp, nullptr, nullptr), HJ_ERR_INVALID_ARG);

    // variable coefficients and the adjoint
    hj_vc_problem vp;
    std::memset(&vp, 0, sizeof vp);
    vp.nx = vp.ny = 16;
    vp.ld = 16;
    vp.lda = 18;
    vp.hx = vp.hy = 1.0 / 17;
    vp.a = (const double *)FAKE;
    vp.batch = 1;
    hj_vc_problem bvp = vp;
    bvp.lda = 17;
    EXPECT(hj_solve_vc_2d(&bvp, (const double *)FAKE, (double *)FAKE, &p, nullptr, &info), HJ_ERR_INVALID_ARG);
    EXPECT(hj_vc_grad_a(&vp, (const double *)FAKE, (const double *)FAKE, (double *)FAKE, 17, nullptr),
           HJ_ERR_INVALID_ARG);
    EXPECT(hj_solve_adjoint(nullptr, nullptr, nullptr), HJ_ERR_INVALID_ARG);
    hj_adjoint_desc d;
    std::memset(&d, 0, sizeof d);
    d.prob = vp;
    d.dl_du = (const double *)FAKE;
    d.lam = (double *)FAKE;
    d.dl_da = (double *)FAKE;  // a gradient without forward states
    d.ld_grad = 18;
    d.params = p;
    EXPECT(hj_solve_adjoint(&d, nullptr, &info), HJ_ERR_INVALID_ARG);

    // helpers
    if (hj_axis_tiles(0, 32, 0) != -1 || hj_axis_tiles(100, 32, 4) != 4) ++failures;
    if (!hj_status_string(HJ_ERR_HIP) || !hj_version()) ++failures;
    if (std::strcmp(hj_status_string((hj_status)77), "HJ_ERR_UNKNOWN") != 0) ++failures;
    if (std::strcmp(hj_status_string((hj_status)-5), "HJ_ERR_UNKNOWN") != 0) ++failures;
    EXPECT(hj_solve_2d(8, 8, 8, 0.1, 0.1, (hj_dtype)-1, FAKE, FAKE, &p, nullptr, &info), HJ_ERR_INVALID_ARG);
    EXPECT(hj_residual(2, 8, 8, 8, 0.1, 0.1, (hj_dtype)123456, FAKE, FAKE, nullptr, &nrm, nullptr),
           HJ_ERR_INVALID_ARG);
    // right-hand-side tuner
    {
        hj_tune_params t;
        std::memset(&t, 0, sizeof t);
        t.trial_tol = 1e-4;
        t.max_trial_cycles = 100;
        hj_params best;
        double ms = 0.0;
        auto tune = [&](const hj_tune_params *tp, int64_t ld) {
            return hj_autotune_solve(64, 64, ld, 0.01, 0.01, HJ_F64, FAKE, FAKE, tp, nullptr, &best, &ms);
        };
        EXPECT(tune(nullptr, 64), HJ_ERR_INVALID_ARG);
        hj_tune_params u = t;
        u.trial_tol = 0.0;
        EXPECT(tune(&u, 64), HJ_ERR_INVALID_ARG);
        u = t;
        u.nrhs = -3;
        EXPECT(tune(&u, 64), HJ_ERR_INVALID_ARG);
        u = t;
        u.nrhs = 2;
        u.rhs_stride = 64 * 64 - 1;
        EXPECT(tune(&u, 64), HJ_ERR_INVALID_ARG);
        u.rhs_stride = (int64_t)1 << 62;  // ny * ld would overflow int64
        EXPECT(tune(&u, (int64_t)1 << 60), HJ_ERR_INVALID_ARG);
    }

    std::printf("libhj validation sanitizer run: %d failures\n", failures);
    return failures ? 1 : 0;
}
