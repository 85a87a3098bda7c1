// hj_api.hip -- C ABI of libhj: argument validation, per-device scratch, and
// the host loop that enqueues cycles and polls the device-side convergence
// flag (declarations and contracts in include/hj.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>
#include <string>

#include "hj.h"
#include "hj_launch.h"

namespace {

thread_local std::string g_err;

hj_status fail(hj_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

hj_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return HJ_ERR_HIP;
}

#define HJ_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- scratch
// One set per device: a second iterate array, reduction partials, the control
// block and two pinned host slots for polling it.  Grown on demand, kept until
// the process ends.  The mutex serialises calls on one device.
struct DevScratch {
    std::mutex mu;
    bool ready = false;
    void *xbuf = nullptr;
    size_t xbytes = 0;
    double *partials = nullptr;
    int64_t npart = 0;
    void *rbuf = nullptr;  // mixed precision: FP32 residual and correction
    size_t rbytes = 0;
    hj::Ctrl *ctrl = nullptr;
    hj::Ctrl *host = nullptr;  // 2 pinned slots
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t tev[2] = {nullptr, nullptr};  // timing events of the autotuner
};

constexpr int kMaxDev = 64;
DevScratch g_scr[kMaxDev];

hj_status scratch_ensure(DevScratch &S, size_t xbytes, int64_t npart, size_t rbytes = 0)
{
    if (!S.ready) {
        HJ_HIP(hipMalloc((void **)&S.ctrl, sizeof(hj::Ctrl)));
        HJ_HIP(hipHostMalloc((void **)&S.host, 2 * sizeof(hj::Ctrl), hipHostMallocDefault));
        HJ_HIP(hipEventCreateWithFlags(&S.ev[0], hipEventDisableTiming));
        HJ_HIP(hipEventCreateWithFlags(&S.ev[1], hipEventDisableTiming));
        S.ready = true;
    }
    if (xbytes > S.xbytes) {
        if (S.xbuf) HJ_HIP(hipFree(S.xbuf));
        S.xbuf = nullptr;
        S.xbytes = 0;
        HJ_HIP(hipMalloc(&S.xbuf, xbytes));
        S.xbytes = xbytes;
    }
    if (rbytes > S.rbytes) {
        if (S.rbuf) HJ_HIP(hipFree(S.rbuf));
        S.rbuf = nullptr;
        S.rbytes = 0;
        HJ_HIP(hipMalloc(&S.rbuf, rbytes));
        S.rbytes = rbytes;
    }
    if (npart > S.npart) {
        if (S.partials) HJ_HIP(hipFree(S.partials));
        S.partials = nullptr;
        S.npart = 0;
        HJ_HIP(hipMalloc((void **)&S.partials, (size_t)npart * sizeof(double)));
        S.npart = npart;
    }
    return HJ_OK;
}

// ---------------------------------------------------------------- validation
size_t esize(hj_dtype dt) { return dt == HJ_F64 ? 8 : 4; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

hj_status check_ptr_dtype(const void *p, hj_dtype dt, const char *name, bool may_be_null)
{
    if (!p) return may_be_null ? HJ_OK : fail(HJ_ERR_INVALID_ARG, std::string(name) + " is NULL");
    if ((uintptr_t)p % esize(dt))
        return fail(HJ_ERR_INVALID_ARG, std::string(name) + " is not aligned to the element size");
    return HJ_OK;
}

hj_status check_params(const hj_params *p, int dim)
{
    if (!p) return fail(HJ_ERR_INVALID_ARG, "params is NULL");
    if (p->flags & ~(HJ_FLAG_LDS_KERNEL | HJ_FLAG_LAUNCH_PER_CYCLE))
        return fail(HJ_ERR_INVALID_ARG, "unknown bits in params.flags");
    if (p->method != HJ_HIERARCHICAL && p->method != HJ_GLOBAL)
        return fail(HJ_ERR_INVALID_ARG, "params.method must be HJ_HIERARCHICAL or HJ_GLOBAL");
    if (p->max_cycles < 1) return fail(HJ_ERR_INVALID_ARG, "params.max_cycles must be >= 1");
    if (p->check_every < 0) return fail(HJ_ERR_INVALID_ARG, "params.check_every must be >= 0");
    if (std::isnan(p->rel_tol)) return fail(HJ_ERR_INVALID_ARG, "params.rel_tol is NaN");
    if (p->method == HJ_HIERARCHICAL) {
        if (p->s < 1) return fail(HJ_ERR_INVALID_ARG, "params.s must be >= 1");
        const int tx = p->tile_x ? p->tile_x : 32;
        const int ty = p->tile_y ? p->tile_y : 32;
        if (tx < 1 || (dim == 2 && ty < 1)) return fail(HJ_ERR_INVALID_ARG, "tile extents must be >= 1");
        if (p->overlap_x < 0 || p->overlap_x >= tx)
            return fail(HJ_ERR_INVALID_ARG, "params.overlap_x must satisfy 0 <= overlap_x < tile_x");
        if (dim == 2 && (p->overlap_y < 0 || p->overlap_y >= ty))
            return fail(HJ_ERR_INVALID_ARG, "params.overlap_y must satisfy 0 <= overlap_y < tile_y");
        if (dim == 2 && !hj::cycle2d_supported(tx, ty))
            return fail(HJ_ERR_UNSUPPORTED,
                        "2D tile shape not provided (tile_x, tile_y in {16, 32, 64, 128}; "
                        "tile_x = 16 only with tile_y <= 64)");
        if (dim == 1 && !hj::cycle1d_supported(tx))
            return fail(HJ_ERR_UNSUPPORTED, "1D tile not provided (32, 64, ..., 1024)");
    }
    return HJ_OK;
}

// Device pointers must live on the current device (a host pointer handed to a
// kernel would fault).
hj_status check_device_ptr(const void *p, int dev, const char *name)
{
    if (!p) return HJ_OK;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HJ_ERR_INVALID_ARG, std::string(name) + " is not device memory");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(HJ_ERR_INVALID_ARG, std::string(name) + " is not device memory");
    if (a.device != dev)
        return fail(HJ_ERR_INVALID_ARG, std::string(name) + " lives on another device");
    return HJ_OK;
}

// ---------------------------------------------------------------- driver
// Iterates rotate through three arrays (the caller's x and two scratch
// arrays): cycle c reads bufs[c % 3] and writes bufs[(c + 1) % 3].  The verdict
// on iterate c is reached inside cycle kernel c + 1, which is still allowed to
// run, so the converged iterate must survive two more writes.
struct Step {
    // one cycle xin -> xout; res: fused residual of xin under red
    std::function<hipError_t(const void *, void *, bool, double, const hj::Red &)> cycle;
    // residual of x, partial sums into part
    std::function<hipError_t(const void *, double *)> resid;
    // copy an iterate into the caller's x
    std::function<hipError_t(void *, const void *)> copy;
    int nb_cycle;  // workgroups of one cycle kernel
    int nb_resid;  // workgroups of the residual kernel
};

// Where a solve keeps its device control block and reduction partials, and how
// the host reads the block: through two pinned slots and events (one batch of
// lookahead), or, without them (host == nullptr), by a copy into host memory
// after each batch followed by a stream synchronisation.
struct Ctl {
    hj::Ctrl *ctrl;
    double *partials;  // npart doubles: two halves, by cycle parity
    int64_t npart;
    hj::Ctrl *host;    // 2 pinned slots, or nullptr
    hipEvent_t ev[2];
};

Ctl ctl_of(DevScratch &S) { return Ctl{S.ctrl, S.partials, S.npart, S.host, {S.ev[0], S.ev[1]}}; }

hj_status read_ctrl(const Ctl &K, hipStream_t stream, hj::Ctrl &c)
{
    if (K.host) {
        HJ_HIP(hipMemcpyAsync(&K.host[0], K.ctrl, sizeof(hj::Ctrl), hipMemcpyDeviceToHost, stream));
        HJ_HIP(hipStreamSynchronize(stream));
        c = K.host[0];
    } else {
        HJ_HIP(hipMemcpyAsync(&c, K.ctrl, sizeof(hj::Ctrl), hipMemcpyDeviceToHost, stream));
        HJ_HIP(hipStreamSynchronize(stream));
    }
    return HJ_OK;
}

hj_status read_ctrl(DevScratch &S, hipStream_t stream, hj::Ctrl &c) { return read_ctrl(ctl_of(S), stream, c); }

// latest: in tolerance mode, hand back iterate c + 1 instead of the first
// iterate c that met the tolerance: it is whole (see stopped()) and one cycle
// further on; callers that only need a good iterate (the refinement phases)
// take it, info->cycles then counts it.
// sw_tol >= 0: the solve may end early at the hand-over point of Ctrl
// (relative residual <= sw_tol reached first at a cycle >= sw_min_c); it
// then returns HJ_OK with *status_out = ST_SWITCH and iterate c + 1.
hj_status drive(const Step &st, void *xu, void *xs, size_t xbytes, const hj_params &p, int64_t spc,
                hipStream_t stream, const Ctl &S, hj_info *info, bool latest = false,
                double sw_tol = -1.0, int64_t sw_min_c = 0, int32_t *status_out = nullptr)
{
    void *bufs[3] = {xu, xs, (char *)xs + xbytes};
    double *part[2] = {S.partials, S.partials + S.npart / 2};
    const int64_t maxc = p.max_cycles;
    hj_status r;
    HJ_HIP(hj::launch_ctrl_init(S.ctrl, stream, p.rel_tol > 0.0 ? sw_tol : -1.0, sw_min_c));
    int64_t final_c = maxc;
    hj::Ctrl c{};
    if (p.rel_tol <= 0.0) {
        // fixed count: residuals of x_0 and x_maxc only
        HJ_HIP(st.resid(bufs[0], part[0]));
        HJ_HIP(hj::launch_judge(part[0], st.nb_resid, S.ctrl, 0, -1.0, stream));
        const hj::Red none{nullptr, nullptr, S.ctrl, 0, 0};
        for (int64_t k = 0; k < maxc; ++k)
            HJ_HIP(st.cycle(bufs[k % 3], bufs[(k + 1) % 3], false, -1.0, none));
        HJ_HIP(st.resid(bufs[maxc % 3], part[1]));
        HJ_HIP(hj::launch_judge(part[1], st.nb_resid, S.ctrl, maxc, -1.0, stream));
        if ((r = read_ctrl(S, stream, c)) != HJ_OK) return r;
    } else {
        const double tol = p.rel_tol;
        int64_t next = 0;
        // check_every > 0: fixed batch.  0: batches sized to about kBatchUs of
        // GPU time from the cycle rate observed between polls, so that at most
        // a batch or two of early-exit launches follow convergence.
        constexpr double kBatchUs = 500.0;
        int64_t batch = p.check_every > 0 ? p.check_every : 4;
        auto launch_batch = [&]() -> hj_status {
            const int64_t k = std::min<int64_t>(batch, maxc - next);
            for (int64_t i = 0; i < k; ++i) {
                const int64_t cc = next + i;
                const hj::Red red{part[cc & 1], part[(cc + 1) & 1], S.ctrl, cc, cc > 0 ? st.nb_cycle : 0};
                HJ_HIP(st.cycle(bufs[cc % 3], bufs[(cc + 1) % 3], true, tol, red));
            }
            next += k;
            return HJ_OK;
        };
        auto t_prev = std::chrono::steady_clock::now();
        int64_t iter_prev = 0;
        auto adapt = [&](int64_t iter_now) {
            if (p.check_every != 0) return;
            const auto t_now = std::chrono::steady_clock::now();
            const int64_t done = iter_now - iter_prev;
            const double us = std::chrono::duration<double, std::micro>(t_now - t_prev).count();
            if (done > 0 && us > 0.0) {
                const double per = us / (double)done;
                batch = std::max<int64_t>(4, std::min<int64_t>(256, (int64_t)(kBatchUs / per)));
            }
            t_prev = t_now;
            iter_prev = iter_now;
        };
        if (S.host) {
            // one batch of lookahead: the next batch is enqueued before the
            // host waits for the control block copied after the current one
            auto enqueue = [&](int slot) -> hj_status {
                hj_status e;
                if ((e = launch_batch()) != HJ_OK) return e;
                S.host[slot].iter = -1;
                HJ_HIP(hipMemcpyAsync(&S.host[slot], S.ctrl, sizeof(hj::Ctrl), hipMemcpyDeviceToHost, stream));
                HJ_HIP(hipEventRecord(S.ev[slot], stream));
                return HJ_OK;
            };
            if ((r = enqueue(0)) != HJ_OK) return r;
            int slot = 0;
            for (;;) {
                const bool more = next < maxc;
                if (more && (r = enqueue(slot ^ 1)) != HJ_OK) return r;  // keep the GPU fed
                HJ_HIP(hipEventSynchronize(S.ev[slot]));
                if (S.host[slot].status != hj::ST_RUNNING || !more) break;
                adapt(S.host[slot].iter);
                slot ^= 1;
            }
        } else {
            // no pinned slots or events: the stream drains after every batch
            for (;;) {
                if ((r = launch_batch()) != HJ_OK) return r;
                if ((r = read_ctrl(S, stream, c)) != HJ_OK) return r;
                if (c.status != hj::ST_RUNNING || next >= maxc) break;
                adapt(c.iter);
            }
        }
        if ((r = read_ctrl(S, stream, c)) != HJ_OK) return r;
        if (c.status == hj::ST_RUNNING) {
            // every cycle ran: judge the last two iterates here
            HJ_HIP(hj::launch_judge(part[(maxc - 1) & 1], st.nb_cycle, S.ctrl, maxc - 1, tol, stream));
            HJ_HIP(st.resid(bufs[maxc % 3], part[maxc & 1]));
            HJ_HIP(hj::launch_judge(part[maxc & 1], st.nb_resid, S.ctrl, maxc, tol, stream));
            if ((r = read_ctrl(S, stream, c)) != HJ_OK) return r;
        }
        final_c = c.status != hj::ST_RUNNING ? c.done_cycle : maxc;
        if ((latest && c.status == hj::ST_CONVERGED) || c.status == hj::ST_SWITCH)
            final_c = std::min<int64_t>(c.done_cycle + 1, maxc);
    }
    if (status_out) *status_out = c.status;
    if (final_c % 3 != 0) {
        HJ_HIP(st.copy(xu, bufs[final_c % 3]));
        HJ_HIP(hipStreamSynchronize(stream));
    }
    if (info) {
        info->cycles = final_c;
        info->sweeps = final_c * spc;
        info->r0_norm = std::sqrt(c.r0sq);
        info->rel_residual = c.r0sq > 0.0 ? std::sqrt(c.last_rsq) / std::sqrt(c.r0sq) : 0.0;
        if (!std::isfinite(c.last_rsq)) info->rel_residual = NAN;
    }
    if (c.status == hj::ST_NONFINITE) return fail(HJ_ERR_NONFINITE, "residual norm became non-finite");
    if (p.rel_tol > 0.0 && c.status != hj::ST_CONVERGED && c.status != hj::ST_SWITCH)
        return fail(HJ_ERR_NOT_CONVERGED, "max_cycles reached before rel_tol");
    return HJ_OK;
}

constexpr const char *kNeedFullTile =
    "tiles with a 128 extent run only in the register kernel, on grids of at least one full tile "
    "(nx >= tile_x, ny >= tile_y, no HJ_FLAG_LDS_KERNEL)";

hj::Geom2 make_geom2(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, const hj_params &p)
{
    hj::Geom2 g;
    g.nx = (int)nx;
    g.ny = (int)ny;
    g.ld = ld;
    g.tx = p.tile_x ? p.tile_x : 32;
    g.ty = p.tile_y ? p.tile_y : 32;
    g.ox = p.overlap_x;
    g.oy = p.overlap_y;
    g.ntx = hj::axis_count(g.nx, g.tx, g.ox);
    g.nty = hj::axis_count(g.ny, g.ty, g.oy);
    g.iso = hx == hy;
    g.reg = (p.flags & HJ_FLAG_LDS_KERNEL) ? 0 : 1;
    g.hh = hx * hx;
    g.wx = 1.0 / (hx * hx);
    g.wy = 1.0 / (hy * hy);
    g.dinv = 1.0 / (2.0 * g.wx + 2.0 * g.wy);
    return g;
}

hj::Geom1 make_geom1(int64_t n, double h, const hj_params *p)
{
    hj::Geom1 g;
    g.n = n;
    g.t = p && p->tile_x ? p->tile_x : 32;
    g.o = p ? p->overlap_x : 0;
    g.nt = hj::axis_count((int)n, g.t, g.o);
    g.hh = h * h;
    g.w1 = 1.0 / (h * h);
    return g;
}

constexpr int64_t kMaxAxis = (int64_t)1 << 30;

hj_status check_vc_problem(const hj_vc_problem *pr)
{
    if (!pr) return fail(HJ_ERR_INVALID_ARG, "problem is NULL");
    if (pr->nx < 1 || pr->ny < 1 || pr->nx > kMaxAxis || pr->ny > kMaxAxis)
        return fail(HJ_ERR_INVALID_ARG, "nx, ny must be in [1, 2^30]");
    if (pr->ld < pr->nx) return fail(HJ_ERR_INVALID_ARG, "ld must be >= nx");
    if (pr->lda < pr->nx + 2) return fail(HJ_ERR_INVALID_ARG, "lda must be >= nx + 2");
    if (!finite_pos(pr->hx) || !finite_pos(pr->hy)) return fail(HJ_ERR_INVALID_ARG, "hx, hy must be finite and > 0");
    if (pr->batch < 1) return fail(HJ_ERR_INVALID_ARG, "batch must be >= 1");
    if (pr->flags != 0) return fail(HJ_ERR_INVALID_ARG, "problem flags must be 0");
    if (pr->batch > 1 && pr->batch_stride < pr->ny * pr->ld)
        return fail(HJ_ERR_INVALID_ARG, "batch_stride must be >= ny * ld");
    return check_ptr_dtype(pr->a, HJ_F64, "a", false);
}

hj::GeomVC make_geom_vc(const hj_vc_problem &pr, const hj_params &p)
{
    hj::GeomVC g;
    g.nx = (int)pr.nx;
    g.ny = (int)pr.ny;
    g.ld = pr.ld;
    g.tx = p.tile_x ? p.tile_x : 32;
    g.ty = p.tile_y ? p.tile_y : 32;
    g.ox = p.overlap_x;
    g.oy = p.overlap_y;
    g.ntx = hj::axis_count(g.nx, g.tx, g.ox);
    g.nty = hj::axis_count(g.ny, g.ty, g.oy);
    g.a = pr.a;
    g.lda = pr.lda;
    g.ihx2 = 1.0 / (pr.hx * pr.hx);
    g.ihy2 = 1.0 / (pr.hy * pr.hy);
    g.reg = (p.flags & HJ_FLAG_LDS_KERNEL) ? 0 : 1;
    return g;
}

hj_status solve_vc_locked(const hj_vc_problem &pr, const double *f, double *u, const hj_params &P,
                          hipStream_t st, DevScratch &S, hj_info *infos)
{
    const hj::GeomVC g = make_geom_vc(pr, P);
    const bool hier = P.method == HJ_HIERARCHICAL;
    const int64_t nbc = hier ? hj::cycle_vc_blocks(g) : hj::sweep_vc_blocks(g);
    const int64_t nbr = hj::sweep_vc_blocks(g);
    if (nbc > INT32_MAX || nbr > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "grid too large");
    const size_t xbytes = (size_t)pr.ny * (size_t)pr.ld * 8;
    hj_status r;
    if ((r = scratch_ensure(S, 2 * xbytes, 2 * std::max(nbc, nbr))) != HJ_OK) return r;
    hj_status worst = HJ_OK;
    for (int b = 0; b < pr.batch; ++b) {
        const double *fb = f + (int64_t)b * pr.batch_stride;
        double *ub = u + (int64_t)b * pr.batch_stride;
        Step step;
        step.nb_cycle = (int)nbc;
        step.nb_resid = (int)nbr;
        step.cycle = [&](const void *xi, void *xo, bool res, double tol, const hj::Red &red) {
            return hier ? hj::launch_cycle_vc(g, P.s, res, fb, (const double *)xi, (double *)xo, red, tol, st)
                        : hj::launch_sweep_vc(g, res, fb, (const double *)xi, (double *)xo, red, tol, st);
        };
        step.resid = [&](const void *xi, double *part) {
            return hj::launch_resid_vc(g, fb, (const double *)xi, nullptr, part, st);
        };
        step.copy = [&](void *dst, const void *src) {
            return hipMemcpy2DAsync(dst, (size_t)pr.ld * 8, src, (size_t)pr.ld * 8, (size_t)pr.nx * 8,
                                    (size_t)pr.ny, hipMemcpyDeviceToDevice, st);
        };
        const hj_status sb = drive(step, ub, S.xbuf, xbytes, P, hier ? P.s : 1, st, ctl_of(S),
                                   infos ? &infos[b] : nullptr);
        if (sb == HJ_ERR_HIP || sb == HJ_ERR_INVALID_ARG) return sb;
        if (sb != HJ_OK && worst == HJ_OK) worst = sb;
    }
    return worst;
}


// ---------------------------------------------------------------- batches
// Per-device scratch of hj_solve_batched: one iterate array per problem in a
// single arena, the device problem table, work lists, partials, control
// blocks, the cycle counter, pinned host copies of the control blocks, and a
// stream to capture the cycle graph on.  Grown on demand, guarded by the
// device's mutex.
struct BatchScratch {
    hipStream_t cap = nullptr;
    void *arena = nullptr;
    int64_t arena_bytes = 0;
    hj::BProb *probs = nullptr;
    int64_t nprobs = 0;
    int32_t *owner = nullptr;
    int64_t nowner = 0;
    double *part = nullptr;
    int64_t npart = 0;
    hj::BState *state = nullptr;
    int64_t nstate = 0;
    hj::BState *host = nullptr;  // 2 x nhost pinned
    int64_t nhost = 0;
    void *wg = nullptr;  // one-workgroup 1D batches: problem table and states
    size_t wg_bytes = 0;
};

BatchScratch g_bat[kMaxDev];

template <typename T>
hj_status grow_dev(T *&ptr, int64_t &have, int64_t need)
{
    if (need <= have) return HJ_OK;
    if (ptr) HJ_HIP(hipFree(ptr));
    ptr = nullptr;
    have = 0;
    HJ_HIP(hipMalloc((void **)&ptr, (size_t)need * sizeof(T)));
    have = need;
    return HJ_OK;
}

// ---------------------------------------------------------------- autotuner
using TuneKey = std::tuple<int, int64_t, int64_t, int, int, int>;  // dim, nx, ny, dtype, tx max, ty max
std::map<TuneKey, std::pair<hj_params, double>> g_tune[kMaxDev];

// Time one cycle shape on a zero problem (values do not change the timing:
// no subnormals arise).  Returns microseconds per cycle, or a negative value
// when the shape cannot run on this grid.
hj_status time_shape(int dim, int64_t nx, int64_t ny, hj_dtype dt, const hj_params &P, void *f,
                     void *xa, void *xb, hipStream_t st, DevScratch &S, double &us)
{
    const int idt = dt == HJ_F64 ? hj::F64 : hj::F32;
    const hj::Red none{nullptr, nullptr, S.ctrl, 0, 0};
    const double h = 1.0 / (double)(nx + 1);
    hj::Geom2 g2{};
    hj::Geom1 g1{};
    if (dim == 2) {
        g2 = make_geom2(nx, ny, nx, h, h, P);
        if (!g2.reg || nx < g2.tx || ny < g2.ty) {
            us = -1.0;
            return HJ_OK;
        }
    } else {
        g1 = make_geom1(nx, h, &P);
    }
    auto run = [&](int k) -> hipError_t {
        for (int i = 0; i < k; ++i) {
            const void *src = (i & 1) ? xb : xa;
            void *dst = (i & 1) ? xa : xb;
            const hipError_t e = dim == 2 ? hj::launch_cycle2d(idt, g2, P.s, false, f, src, dst, none, -1.0, st)
                                          : hj::launch_cycle1d(idt, g1, P.s, false, f, src, dst, none, -1.0, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    HJ_HIP(run(1));  // warm-up
    int k = 2;
    for (int pass = 0; pass < 2; ++pass) {
        HJ_HIP(hipEventRecord(S.tev[0], st));
        HJ_HIP(run(k));
        HJ_HIP(hipEventRecord(S.tev[1], st));
        HJ_HIP(hipEventSynchronize(S.tev[1]));
        float ms = 0.0f;
        HJ_HIP(hipEventElapsedTime(&ms, S.tev[0], S.tev[1]));
        us = 1e3 * (double)ms / k;
        // second pass long enough to average out launch jitter (about 1 ms)
        k = (int)std::min(64.0, std::max(3.0, 1000.0 / std::max(us, 1.0)));
    }
    return HJ_OK;
}

// Points a cycle's tiles load per grid point along both axes (1: no
// redundancy).  Tuners skip shapes that load more than kMaxLoadFactor times
// the grid: a cycle's cost grows with that factor and its sweeps with s <=
// 32 at most, so such a shape takes at least twice as long per classical
// sweep as the compact ones (about 0.15 of a load per sweep), while timing
// it (tiles every two points, say) costs more than all other candidates.
constexpr double kMaxLoadFactor = 8.0;

double load_factor(int64_t nx, int64_t ny, int tx, int ty, int ox, int oy)
{
    auto axis = [](int64_t n, int t, int o) {
        return (double)hj::axis_count((int)n, t, o) * (double)std::min<int64_t>(n, t) / (double)n;
    };
    return axis(nx, tx, ox) * (ny > 1 ? axis(ny, ty, oy) : 1.0);
}

hj_status autotune_locked(int dim, int64_t nx, int64_t ny, hj_dtype dt, int txmax, int tymax,
                          hipStream_t st, int dev, DevScratch &S, hj_params &best, double &best_us)
{
    const TuneKey key{dim, nx, ny, (int)dt, txmax, tymax};
    auto it = g_tune[dev].find(key);
    if (it != g_tune[dev].end()) {
        best = it->second.first;
        best_us = it->second.second;
        return HJ_OK;
    }
    const int64_t npts = dim == 2 ? nx * ny : nx;
    const size_t bytes = (size_t)npts * esize(dt);
    hj_status r;
    if ((r = scratch_ensure(S, 3 * bytes, 2)) != HJ_OK) return r;
    if (!S.tev[0]) {
        HJ_HIP(hipEventCreate(&S.tev[0]));
        HJ_HIP(hipEventCreate(&S.tev[1]));
    }
    char *base = (char *)S.xbuf;
    HJ_HIP(hipMemsetAsync(base, 0, 3 * bytes, st));
    void *f = base, *xa = base + bytes, *xb = base + 2 * bytes;

    std::vector<hj_params> cands;
    auto add = [&](int tx, int ty, int s) {
        hj_params P;
        hj_params_default(&P);
        P.tile_x = tx;
        P.tile_y = dim == 2 ? ty : 0;
        P.s = s;
        P.overlap_x = 2 * s - 2;
        P.overlap_y = dim == 2 ? 2 * s - 2 : 0;
        if (load_factor(nx, ny, tx, dim == 2 ? ty : 1, P.overlap_x, P.overlap_y) > kMaxLoadFactor) return;
        cands.push_back(P);
    };
    if (dim == 2) {
        const int shapes[][2] = {{32, 32}, {64, 32}, {32, 64}, {64, 64}, {32, 128}, {64, 128}};
        for (auto &sh : shapes) {
            if (sh[0] > txmax || sh[1] > tymax || sh[0] > nx || sh[1] > ny) continue;
            for (int s : {4, 6, 8, 10, 12, 16})
                if (2 * s - 2 <= std::min(sh[0], sh[1]) - 2) add(sh[0], sh[1], s);
        }
    } else {
        for (int t : {64, 128, 256, 512, 1024}) {
            if (t > txmax || (t > nx && t != 64)) continue;
            for (int s : {4, 8, 12, 16, 24, 32})
                if (2 * s - 2 <= t - 2) add(t, 0, s);
        }
    }
    if (cands.empty())
        return fail(HJ_ERR_UNSUPPORTED, dim == 2 ? "autotune: the grid is smaller than a 32 x 32 tile"
                                                 : "autotune: no 1D tile fits");
    best_us = INFINITY;
    for (const hj_params &P : cands) {
        double us = 0.0;
        if ((r = time_shape(dim, nx, ny, dt, P, f, xa, xb, st, S, us)) != HJ_OK) return r;
        if (us <= 0.0) continue;
        const double per_sweep = us / P.s;
        if (per_sweep < best_us) {
            best_us = per_sweep;
            best = P;
        }
    }
    if (!std::isfinite(best_us)) return fail(HJ_ERR_UNSUPPORTED, "autotune: no candidate runs on this grid");
    g_tune[dev][key] = {best, best_us};
    return HJ_OK;
}

// Shapes for a batch: 2D tuned on its largest problem with tiles that fit
// the smallest (tile_x <= 64, the batched kernel's widths); 1D on its largest.
hj_status tune_batch_locked(const hj_problem *probs, int64_t nprob, hj_dtype dt, hipStream_t st, int dev,
                            DevScratch &S, hj_params &P2, hj_params &P1)
{
    int64_t min_nx = INT64_MAX, min_ny = INT64_MAX, big2 = -1, big1 = -1;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj_problem &q = probs[i];
        if (q.dim == 2) {
            min_nx = std::min(min_nx, q.nx);
            min_ny = std::min(min_ny, q.ny);
            if (big2 < 0 || q.nx * q.ny > probs[big2].nx * probs[big2].ny) big2 = i;
        } else if (big1 < 0 || q.nx > probs[big1].nx) {
            big1 = i;
        }
    }
    hj_status r;
    double us = 0.0;
    if (big2 >= 0 &&
        (r = autotune_locked(2, probs[big2].nx, probs[big2].ny, dt, (int)std::min<int64_t>(min_nx, 64),
                             (int)std::min<int64_t>(min_ny, 128), st, dev, S, P2, us)) != HJ_OK)
        return r;
    if (big1 >= 0 && (r = autotune_locked(1, probs[big1].nx, 1, dt, 1 << 30, 1 << 30, st, dev, S, P1, us)) != HJ_OK)
        return r;
    return HJ_OK;
}

hj_status check_problem(const hj_problem &q, hj_dtype dt, int dev, int64_t i)
{
    const std::string at = "problem " + std::to_string(i) + ": ";
    if (q.flags != 0) return fail(HJ_ERR_INVALID_ARG, at + "flags must be 0");
    if (q.dim != 1 && q.dim != 2) return fail(HJ_ERR_INVALID_ARG, at + "dim must be 1 or 2");
    if (q.nx < 1 || q.nx > kMaxAxis) return fail(HJ_ERR_INVALID_ARG, at + "nx must be in [1, 2^30]");
    if (!finite_pos(q.hx)) return fail(HJ_ERR_INVALID_ARG, at + "hx must be finite and > 0");
    if (q.dim == 2) {
        if (q.ny < 1 || q.ny > kMaxAxis) return fail(HJ_ERR_INVALID_ARG, at + "ny must be in [1, 2^30]");
        if (q.ld < q.nx) return fail(HJ_ERR_INVALID_ARG, at + "ld must be >= nx");
        if (!finite_pos(q.hy)) return fail(HJ_ERR_INVALID_ARG, at + "hy must be finite and > 0");
    }
    hj_status r;
    if ((r = check_ptr_dtype(q.f, dt, (at + "f").c_str(), false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(q.x, dt, (at + "x").c_str(), false)) != HJ_OK) return r;
    if (dev >= 0) {
        if ((r = check_device_ptr(q.f, dev, (at + "f").c_str())) != HJ_OK) return r;
        if ((r = check_device_ptr(q.x, dev, (at + "x").c_str())) != HJ_OK) return r;
    }
    return HJ_OK;
}

// One batched solve of validated, device-resident problems on the scratch
// set B: plain (rf.refine = 0: cycles of precision dt on each problem) or
// refined (FP64 problems; FP32 corrections inside FP64 refinement, each
// problem on its own schedule).  On return B.host[i] holds problem i's state
// and each x its result.  Device and lock held by the caller.
hj_status run_batch(const hj_problem *probs, int64_t nprob, hj_dtype dt, double tol, int64_t max_cycles,
                    const hj::BRefine &rf, const hj_params &P2, const hj_params &P1, int K, hipStream_t st,
                    DevScratch &S, BatchScratch &B, const hj::GeomVC *vc = nullptr)
{
    const int idt = dt == HJ_F64 ? hj::F64 : hj::F32;
    const size_t es = esize(dt);
    const bool refine = rf.refine != 0;
    hj_status r;

    // host tables: problem records, arena offsets (scratch x; refined: FP32
    // residual and two correction buffers, all with the pitch of x)
    auto align = [](int64_t b) { return (b + 255) / 256 * 256; };
    std::vector<hj::BProb> hp((size_t)nprob);
    std::vector<int64_t> off((size_t)nprob * 4, 0);
    int64_t arena = 0, npart = 0;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj_problem &q = probs[i];
        hj::BProb &b = hp[(size_t)i];
        std::memset(&b, 0, sizeof(b));
        b.dim = q.dim;
        b.dt = idt;
        b.f = q.f;
        b.x = q.x;
        int64_t elems = 0;
        if (q.dim == 2) {
            b.g2 = make_geom2(q.nx, q.ny, q.ld, q.hx, q.hy, P2);
            b.nitems = (int64_t)b.g2.ntx * b.g2.nty;
            b.s = P2.s;
            elems = q.ny * q.ld;
        } else if (q.dim == 3) {
            b.gv = *vc;
            b.nitems = hj::cycle_vc_blocks(b.gv);
            b.s = P2.s;
            elems = q.ny * q.ld;
        } else {
            b.g1 = make_geom1(q.nx, q.hx, &P1);
            b.nitems = hj::cycle1d_blocks(b.g1);
            b.s = P1.s;
            elems = q.nx;
        }
        b.part0 = npart;
        npart += b.nitems;
        b.rnitems = refine ? hj::ref_items(q.dim, q.nx, q.ny) : 0;
        b.tol = tol;
        b.max_cycles = max_cycles;
        off[(size_t)i * 4] = arena;
        arena += align(elems * (int64_t)es);
        if (refine)
            for (int k = 1; k < 4; ++k) {
                off[(size_t)i * 4 + k] = arena;
                arena += align(elems * 4);
            }
    }
    if (npart > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "batch too large");

    if (!B.cap) HJ_HIP(hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking));
    if (!S.ev[0]) {
        if ((r = scratch_ensure(S, 0, 0)) != HJ_OK) return r;
    }
    {
        char *a8 = (char *)B.arena;
        int64_t have = B.arena_bytes;
        if ((r = grow_dev(a8, have, arena)) != HJ_OK) return r;
        B.arena = a8;
        B.arena_bytes = have;
    }
    if ((r = grow_dev(B.probs, B.nprobs, nprob)) != HJ_OK) return r;
    if ((r = grow_dev(B.owner, B.nowner, std::max<int64_t>(npart, 1))) != HJ_OK) return r;
    if ((r = grow_dev(B.part, B.npart, std::max<int64_t>(npart, 1))) != HJ_OK) return r;
    if ((r = grow_dev(B.state, B.nstate, nprob)) != HJ_OK) return r;
    if (nprob > B.nhost) {
        if (B.host) HJ_HIP(hipHostFree(B.host));
        B.host = nullptr;
        B.nhost = 0;
        HJ_HIP(hipHostMalloc((void **)&B.host, (size_t)(2 * nprob) * sizeof(hj::BState), hipHostMallocDefault));
        B.nhost = nprob;
    }
    char *base = (char *)B.arena;
    for (int64_t i = 0; i < nprob; ++i) {
        hj::BProb &b = hp[(size_t)i];
        b.s1 = base + off[(size_t)i * 4];
        if (refine) {
            b.r32 = (float *)(base + off[(size_t)i * 4 + 1]);
            b.e0 = (float *)(base + off[(size_t)i * 4 + 2]);
            b.e1 = (float *)(base + off[(size_t)i * 4 + 3]);
        }
    }
    HJ_HIP(hj::launch_batch_init(B.state, (int)nprob, st));

    // Work lists of the problems still running (iso 2D, other 2D, 1D, in
    // that order in one owner array; a problem's items stay contiguous),
    // uploaded with the updated problem records, and a fixed run of K steps
    // captured on them.  Rebuilt when the running
    // problems hold under half of the listed items, so the tail of
    // long-running problems does not pay for launching everyone else's
    // finished tiles.  The caller's stream is idle whenever this runs.
    std::vector<int32_t> own;
    int64_t n_iso = 0, n_gen = 0, n_1d = 0, n_vc = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
    auto rebuild = [&](const hj::BState *snap) -> hj_status {
        own.clear();
        for (int pass = 0; pass < 4; ++pass) {
            const int64_t start = (int64_t)own.size();
            for (int64_t i = 0; i < nprob; ++i) {
                hj::BProb &b = hp[(size_t)i];
                const int kind = b.dim == 1 ? 2 : b.dim == 3 ? 3 : (b.g2.iso ? 0 : 1);
                if (kind != pass || (snap && snap[i].status != hj::ST_RUNNING)) continue;
                b.item0 = (int64_t)own.size() - start;
                own.insert(own.end(), (size_t)b.nitems, (int32_t)i);
            }
            (pass == 0 ? n_iso : pass == 1 ? n_gen : pass == 2 ? n_1d : n_vc) = (int64_t)own.size() - start;
        }
        HJ_HIP(hipMemcpyAsync(B.probs, hp.data(), hp.size() * sizeof(hj::BProb), hipMemcpyHostToDevice, st));
        if (!own.empty())
            HJ_HIP(hipMemcpyAsync(B.owner, own.data(), own.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HJ_HIP(hipStreamSynchronize(st));  // the host tables change on the next rebuild
        cleanup();
        const hj::BatchLaunch Li{B.probs, B.owner, n_iso, B.state, B.part, P2.s};
        const hj::BatchLaunch Lg{B.probs, B.owner + n_iso, n_gen, B.state, B.part, P2.s};
        const hj::BatchLaunch L1{B.probs, B.owner + n_iso + n_gen, n_1d, B.state, B.part, P1.s};
        const hj::BatchLaunch Lv{B.probs, B.owner + n_iso + n_gen + n_1d, n_vc, B.state, B.part, P2.s};
        HJ_HIP(hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal));
        hipError_t ce = hipSuccess;
        for (int k = 0; k < K && ce == hipSuccess; ++k) {
            if (ce == hipSuccess) ce = hj::launch_batch_cycle2d(idt, refine, P2.tile_x, P2.tile_y, true, Li, B.cap);
            if (ce == hipSuccess) ce = hj::launch_batch_cycle2d(idt, refine, P2.tile_x, P2.tile_y, false, Lg, B.cap);
            if (ce == hipSuccess) ce = hj::launch_batch_cycle1d(idt, refine, P1.tile_x, L1, B.cap);
            if (ce == hipSuccess) ce = hj::launch_batch_cycle_vc(P2.tile_x, P2.tile_y, Lv, B.cap);
            if (ce == hipSuccess) ce = hj::launch_batch_judge(B.probs, (int)nprob, B.state, B.part, rf, B.cap);
        }
        const hipError_t ee = hipStreamEndCapture(B.cap, &graph);
        if (ce != hipSuccess) {
            cleanup();
            return hip_fail(ce, "capturing the batch cycle");
        }
        HJ_HIP(ee);
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            cleanup();
            return hip_fail(ie, "hipGraphInstantiate");
        }
        return HJ_OK;
    };
    if ((r = rebuild(nullptr)) != HJ_OK) return r;

    // Steps: a plain problem stops by its judge of iterate max_cycles; a
    // refined one within max_cycles counted cycles plus, per correction
    // solve, a refinement step and at most one cycle that no result counts.
    const int64_t steps = refine ? max_cycles + 3 * (int64_t)rf.max_outer + 8 : max_cycles + 1;
    const int64_t replays = (steps + K - 1) / K;
    int64_t launched = 0;
    auto enqueue = [&](int slot) -> hipError_t {
        hipError_t e = hipGraphLaunch(exec, st);
        if (e == hipSuccess) ++launched;
        if (e == hipSuccess)
            e = hipMemcpyAsync(B.host + (size_t)slot * nprob, B.state, (size_t)nprob * sizeof(hj::BState),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(S.ev[slot], st);
        return e;
    };
    // replay with one replay of lookahead; poll the states in between
    hipError_t le = enqueue(0);
    int slot = 0;
    while (le == hipSuccess) {
        const bool more = launched < replays;
        if (more && (le = enqueue(slot ^ 1)) != hipSuccess) break;
        if ((le = hipEventSynchronize(S.ev[slot])) != hipSuccess) break;
        const hj::BState *snap = B.host + (size_t)slot * nprob;
        int64_t live_items = 0;
        for (int64_t i = 0; i < nprob; ++i)
            if (snap[i].status == hj::ST_RUNNING) live_items += hp[(size_t)i].nitems;
        if (live_items == 0 || !more) break;
        if (2 * live_items < (int64_t)own.size()) {
            // drain the lookahead replay, then rebuild from its newer snapshot
            if ((le = hipEventSynchronize(S.ev[slot ^ 1])) != hipSuccess) break;
            if ((r = rebuild(B.host + (size_t)(slot ^ 1) * nprob)) != HJ_OK) {
                cleanup();
                return r;
            }
            if (launched >= replays) break;
            if ((le = enqueue(0)) != hipSuccess) break;
            slot = 0;
            continue;
        }
        slot ^= 1;
    }
    if (le == hipSuccess) le = hj::launch_batch_finalize(B.probs, (int)nprob, B.state, st);
    if (le == hipSuccess)
        le = hipMemcpyAsync(B.host, B.state, (size_t)nprob * sizeof(hj::BState), hipMemcpyDeviceToHost, st);
    if (le == hipSuccess) le = hipStreamSynchronize(st);
    cleanup();
    if (le != hipSuccess) return hip_fail(le, "batch replay");
    return HJ_OK;
}

// Several right-hand sides of one variable-coefficient operator: each is a
// problem of the batched engine (one launch per cycle for all of them, each
// judged on its own), so every right-hand side gets the iterates and the
// cycle count of its own solve.
hj_status solve_vc_batched(const hj_vc_problem &pr, const double *f, double *u, const hj_params &P,
                           hipStream_t st, int dev, DevScratch &S, hj_info *infos)
{
    if (!hj::batch_vc_supported(P.tile_x ? P.tile_x : 32, P.tile_y ? P.tile_y : 32))
        return fail(HJ_ERR_UNSUPPORTED, "variable-coefficient tile shape");
    const hj::GeomVC g = make_geom_vc(pr, P);
    std::vector<hj_problem> probs((size_t)pr.batch);
    for (int b = 0; b < pr.batch; ++b) {
        hj_problem &q = probs[(size_t)b];
        std::memset(&q, 0, sizeof(q));
        q.dim = 3;
        q.nx = pr.nx;
        q.ny = pr.ny;
        q.ld = pr.ld;
        q.hx = pr.hx;
        q.hy = pr.hy;
        q.f = f + (int64_t)b * pr.batch_stride;
        q.x = u + (int64_t)b * pr.batch_stride;
    }
    hj_params P2 = P, P1;
    P2.tile_x = g.tx;
    P2.tile_y = g.ty;
    hj_params_default(&P1);
    const double tol = P.rel_tol > 0.0 ? P.rel_tol : -1.0;
    BatchScratch &B = g_bat[dev];
    hj_status r;
    if ((r = run_batch(probs.data(), pr.batch, HJ_F64, tol, P.max_cycles, hj::BRefine{}, P2, P1, 8, st, S, B,
                       &g)) != HJ_OK)
        return r;
    hj_status worst = HJ_OK;
    for (int b = 0; b < pr.batch; ++b) {
        const hj::BState &c = B.host[b];
        if (infos) {
            infos[b].cycles = c.used;
            infos[b].sweeps = c.used * P.s;
            infos[b].r0_norm = std::sqrt(c.r0sq);
            infos[b].rel_residual = c.r0sq > 0.0 ? std::sqrt(c.rsq) / std::sqrt(c.r0sq) : 0.0;
            if (!std::isfinite(c.rsq)) infos[b].rel_residual = NAN;
        }
        if (c.status == hj::ST_NONFINITE) worst = HJ_ERR_NONFINITE;
        else if (c.status != hj::ST_CONVERGED && tol > 0.0 && worst == HJ_OK) worst = HJ_ERR_NOT_CONVERGED;
    }
    if (worst == HJ_ERR_NONFINITE) return fail(worst, "residual norm became non-finite");
    if (worst == HJ_ERR_NOT_CONVERGED) return fail(worst, "max_cycles reached before rel_tol");
    return HJ_OK;
}

// Least FP64 cycles to the switch point for hj_solve_2d_refined to hand over
// to FP32 corrections (hj_refine_params.switch_min_cycles = 0).
constexpr int64_t kSwitchMinCycles = 8;

// Arguments of a 2D solve, checked before any HIP call.
hj_status check_solve_2d(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                         const void *f, const void *x, const hj_params *p)
{
    if (nx < 1 || ny < 1 || nx > kMaxAxis || ny > kMaxAxis)
        return fail(HJ_ERR_INVALID_ARG, "nx, ny must be in [1, 2^30]");
    if (ld < nx) return fail(HJ_ERR_INVALID_ARG, "ld must be >= nx");
    if (!finite_pos(hx) || !finite_pos(hy)) return fail(HJ_ERR_INVALID_ARG, "hx, hy must be finite and > 0");
    if (dtype != HJ_F64 && dtype != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    hj_status r;
    if ((r = check_ptr_dtype(f, dtype, "f", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(x, dtype, "x", false)) != HJ_OK) return r;
    if ((r = check_params(p, 2)) != HJ_OK) return r;
    if (p->method == HJ_HIERARCHICAL && !hj::cycle2d_runnable(make_geom2(nx, ny, ld, hx, hy, *p)))
        return fail(HJ_ERR_UNSUPPORTED, kNeedFullTile);
    return HJ_OK;
}

// The current device, and f and x living on it.
hj_status solve_device(const void *f, const void *x, int &dev)
{
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    hj_status r;
    if ((r = check_device_ptr(f, dev, "f")) != HJ_OK) return r;
    return check_device_ptr(x, dev, "x");
}

// One 2D solve on scratch the caller has set up: the two spare iterate arrays
// at xs (2 xbytes) and the control block and partials in K.
hj_status solve_2d_on(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                      const void *f, void *x, const hj_params &P, hipStream_t st, void *xs,
                      const Ctl &K, hj_info *info)
{
    const hj::Geom2 g = make_geom2(nx, ny, ld, hx, hy, P);
    const int dt = dtype == HJ_F64 ? hj::F64 : hj::F32;
    const size_t es = esize(dtype);
    const bool hier = P.method == HJ_HIERARCHICAL;
    const size_t xbytes = (size_t)ny * (size_t)ld * es;
    Step step;
    step.nb_cycle = (int)(hier ? hj::cycle2d_blocks(g) : hj::sweep2d_blocks(g));
    step.nb_resid = (int)hj::resid2d_blocks(g);
    step.cycle = [&](const void *xi, void *xo, bool res, double tol, const hj::Red &red) {
        return hier ? hj::launch_cycle2d(dt, g, P.s, res, f, xi, xo, red, tol, st)
                    : hj::launch_sweep2d(dt, g, res, f, xi, xo, red, tol, st);
    };
    step.resid = [&](const void *xi, double *part) {
        return hj::launch_resid2d(dt, g, f, xi, nullptr, part, st);
    };
    step.copy = [&](void *dst, const void *src) {
        return hipMemcpy2DAsync(dst, (size_t)ld * es, src, (size_t)ld * es, (size_t)nx * es,
                                (size_t)ny, hipMemcpyDeviceToDevice, st);
    };
    return drive(step, x, xs, xbytes, P, hier ? P.s : 1, st, K, info);
}

// Partials (two halves) a 2D solve needs: one per workgroup of its widest kernel.
hj_status solve_2d_partials(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, const hj_params &P,
                            int64_t &npart)
{
    const hj::Geom2 g = make_geom2(nx, ny, ld, hx, hy, P);
    const int64_t nbc = P.method == HJ_HIERARCHICAL ? hj::cycle2d_blocks(g) : hj::sweep2d_blocks(g);
    const int64_t nbr = hj::resid2d_blocks(g);
    if (nbc > INT32_MAX || nbr > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "grid too large");
    npart = 2 * std::max(nbc, nbr);
    return HJ_OK;
}

// ---------------------------------------------------------------- allocation-free 2D solve
// The scratch of hj_solve_2d_noalloc: the control block, the partials and the
// two spare iterate arrays, carved from one array in the library's own code
// object.  Each device holds its own copy; its address comes from
// hipGetSymbolAddress on the first call on that device (in host code the
// name `scratch` is not a device address).
constexpr size_t kNoAllocBytes = (size_t)HJ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocScratch {
    std::mutex mu;
    unsigned char *ptr = nullptr;  // device address of `scratch` on this device
};
NoAllocScratch g_noalloc[kMaxDev];

constexpr size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

void hj_params_default(hj_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tile_x = 32;
    p->tile_y = 32;
    p->s = 16;
    p->method = HJ_HIERARCHICAL;
    p->max_cycles = 1000000;
    p->check_every = 0;
    p->rel_tol = 1e-6;
}

hj_status hj_solve_2d(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                      const void *f, void *x, const hj_params *p, void *stream, hj_info *info)
{
    g_err.clear();
    hj_status r;
    if ((r = check_solve_2d(nx, ny, ld, hx, hy, dtype, f, x, p)) != HJ_OK) return r;
    int64_t npart = 0;
    if ((r = solve_2d_partials(nx, ny, ld, hx, hy, *p, npart)) != HJ_OK) return r;
    int dev = 0;
    if ((r = solve_device(f, x, dev)) != HJ_OK) return r;

    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    const size_t xbytes = (size_t)ny * (size_t)ld * esize(dtype);
    if ((r = scratch_ensure(S, 2 * xbytes, npart)) != HJ_OK) return r;
    return solve_2d_on(nx, ny, ld, hx, hy, dtype, f, x, *p, (hipStream_t)stream, S.xbuf, ctl_of(S), info);
}

hj_status hj_solve_2d_noalloc(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                              const void *f, void *x, const hj_params *p, void *stream, hj_info *info)
{
    g_err.clear();
    hj_status r;
    if ((r = check_solve_2d(nx, ny, ld, hx, hy, dtype, f, x, p)) != HJ_OK) return r;
    int64_t npart = 0;
    if ((r = solve_2d_partials(nx, ny, ld, hx, hy, *p, npart)) != HJ_OK) return r;
    const size_t xbytes = (size_t)ny * (size_t)ld * esize(dtype);
    const size_t off_part = round256(sizeof(hj::Ctrl));
    const size_t off_x = off_part + round256((size_t)npart * sizeof(double));
    const size_t need = off_x + 2 * xbytes;
    if (need > kNoAllocBytes) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "grid needs %zu bytes of scratch (two iterate arrays of ny * ld elements and "
                      "%lld partials); hj_solve_2d_noalloc holds at most %zu",
                      need, (long long)npart, kNoAllocBytes);
        return fail(HJ_ERR_INVALID_ARG, msg);
    }
    int dev = 0;
    if ((r = solve_device(f, x, dev)) != HJ_OK) return r;

    NoAllocScratch &N = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(N.mu);
    if (!N.ptr) {
        void *a = nullptr;
        HJ_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a) return fail(HJ_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        N.ptr = (unsigned char *)a;
    }
    const Ctl K{(hj::Ctrl *)N.ptr, (double *)(N.ptr + off_part), npart, nullptr, {nullptr, nullptr}};
    return solve_2d_on(nx, ny, ld, hx, hy, dtype, f, x, *p, (hipStream_t)stream, N.ptr + off_x, K, info);
}


hj_status hj_solve_2d_refined(int64_t nx, int64_t ny, int64_t ld, double hx, double hy,
                              const double *f, double *x, const hj_refine_params *p,
                              void *stream, hj_refine_info *info)
{
    g_err.clear();
    if (nx < 1 || ny < 1 || nx > kMaxAxis || ny > kMaxAxis)
        return fail(HJ_ERR_INVALID_ARG, "nx, ny must be in [1, 2^30]");
    if (ld < nx) return fail(HJ_ERR_INVALID_ARG, "ld must be >= nx");
    if (!finite_pos(hx) || !finite_pos(hy)) return fail(HJ_ERR_INVALID_ARG, "hx, hy must be finite and > 0");
    hj_status r;
    if ((r = check_ptr_dtype(f, HJ_F64, "f", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(x, HJ_F64, "x", false)) != HJ_OK) return r;
    if (!p) return fail(HJ_ERR_INVALID_ARG, "params is NULL");
    if (p->flags != 0) return fail(HJ_ERR_INVALID_ARG, "refine flags must be 0");
    if (p->switch_min_cycles < 0) return fail(HJ_ERR_INVALID_ARG, "switch_min_cycles must be >= 0");
    if (!(p->rel_tol > 0.0)) return fail(HJ_ERR_INVALID_ARG, "rel_tol must be > 0");
    if (p->max_outer < 1) return fail(HJ_ERR_INVALID_ARG, "max_outer must be >= 1");
    if (!(p->inner.rel_tol > 0.0)) return fail(HJ_ERR_INVALID_ARG, "inner.rel_tol must be > 0");
    if (!(p->switch_tol >= 0.0) || !std::isfinite(p->switch_tol))
        return fail(HJ_ERR_INVALID_ARG, "switch_tol must be finite and >= 0");
    if ((r = check_params(&p->inner, 2)) != HJ_OK) return r;
    if (p->inner.method == HJ_HIERARCHICAL &&
        !hj::cycle2d_runnable(make_geom2(nx, ny, ld, hx, hy, p->inner)))
        return fail(HJ_ERR_UNSUPPORTED, kNeedFullTile);

    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    if ((r = check_device_ptr(f, dev, "f")) != HJ_OK) return r;
    if ((r = check_device_ptr(x, dev, "x")) != HJ_OK) return r;

    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    const hj_params P = p->inner;
    const hj::Geom2 g = make_geom2(nx, ny, ld, hx, hy, P);
    const bool hier = P.method == HJ_HIERARCHICAL;
    const int64_t nbc = hier ? hj::cycle2d_blocks(g) : hj::sweep2d_blocks(g);
    const int64_t nbr = hj::resid2d_blocks(g);
    const int64_t nbm = hj::resid2d_mixed_blocks(g);
    if (nbc > INT32_MAX || nbr > INT32_MAX || nbm > INT32_MAX)
        return fail(HJ_ERR_UNSUPPORTED, "grid too large");
    const size_t b32 = (size_t)ny * (size_t)ld * sizeof(float);
    const size_t b64 = 2 * b32;
    if ((r = scratch_ensure(S, 2 * b64, 2 * std::max(nbc, std::max(nbr, nbm)), 2 * b32)) != HJ_OK)
        return r;
    hipStream_t st = (hipStream_t)stream;
    float *r32 = (float *)S.rbuf;
    float *e32 = (float *)((char *)S.rbuf + b32);

    Step step;  // FP32 cycles on A e = r32
    step.nb_cycle = (int)nbc;
    step.nb_resid = (int)nbr;
    step.cycle = [&](const void *xi, void *xo, bool res, double tol, const hj::Red &red) {
        return hier ? hj::launch_cycle2d(hj::F32, g, P.s, res, r32, xi, xo, red, tol, st)
                    : hj::launch_sweep2d(hj::F32, g, res, r32, xi, xo, red, tol, st);
    };
    step.resid = [&](const void *xi, double *part) {
        return hj::launch_resid2d(hj::F32, g, r32, xi, nullptr, part, st);
    };
    step.copy = [&](void *dst, const void *src) {
        return hipMemcpy2DAsync(dst, (size_t)ld * 4, src, (size_t)ld * 4, (size_t)nx * 4,
                                (size_t)ny, hipMemcpyDeviceToDevice, st);
    };

    // FP64 residual of x into r32; returns ||f - A x||^2
    auto fp64_residual = [&](double &rsq) -> hj_status {
        HJ_HIP(hj::launch_ctrl_init(S.ctrl, st));
        HJ_HIP(hj::launch_resid2d_f64_to_f32(g, f, x, r32, e32, S.partials, st));
        HJ_HIP(hj::launch_judge(S.partials, (int)nbm, S.ctrl, 0, -1.0, st));
        hj::Ctrl c{};
        hj_status rr = read_ctrl(S, st, c);
        if (rr != HJ_OK) return rr;
        rsq = c.last_rsq;
        return HJ_OK;
    };

    // phase 1: FP64 cycles on x down to the switch tolerance
    // Default switch: FP32 rounding plants slow-mode error of about 1e-6 times
    // the residual at the switch; 1e4 rel_tol keeps it well below rel_tol.  In
    // the exact regime (overlap >= 2s - 2, a cycle is s classical sweeps) the
    // FP32 correction solves reach 1e5 rel_tol's targets as fast as FP64 does
    // (measured), so the switch comes a decade earlier there.
    const bool exact = hier && P.overlap_x >= 2 * P.s - 2 && P.overlap_y >= 2 * P.s - 2;
    const double sw = p->switch_tol > 0.0 ? p->switch_tol : std::min(1.0, (exact ? 1e5 : 1e4) * p->rel_tol);
    int64_t fp64_cycles = 0;
    double r0_phase1 = 0.0;
    Step s64;  // FP64 cycles on A x = f
    s64.nb_cycle = (int)nbc;
    s64.nb_resid = (int)nbr;
    s64.cycle = [&](const void *xi, void *xo, bool res, double tol, const hj::Red &red) {
        return hier ? hj::launch_cycle2d(hj::F64, g, P.s, res, f, xi, xo, red, tol, st)
                    : hj::launch_sweep2d(hj::F64, g, res, f, xi, xo, red, tol, st);
    };
    s64.resid = [&](const void *xi, double *part) {
        return hj::launch_resid2d(hj::F64, g, f, xi, nullptr, part, st);
    };
    s64.copy = [&](void *dst, const void *src) {
        return hipMemcpy2DAsync(dst, (size_t)ld * 8, src, (size_t)ld * 8, (size_t)nx * 8,
                                (size_t)ny, hipMemcpyDeviceToDevice, st);
    };
    // The hand-over is taken only if the FP64 cycles needed at least
    // switch_min_cycles to reach the switch point: about as many remain from
    // there to rel_tol (equal decades on either side in the exact regime), and
    // below that the refinement's own passes (two residuals, the
    // accumulation, a cycle handed over per phase) cost more than FP32 cycles
    // save; such a solve just runs on in FP64 to rel_tol, unchanged.
    if (sw < 1.0) {
        hj_params P64 = P;
        P64.rel_tol = p->rel_tol;
        hj_info i64{};
        int32_t st1 = hj::ST_RUNNING;
        const int64_t kmin = p->switch_min_cycles > 0 ? p->switch_min_cycles : kSwitchMinCycles;
        const hj_status s1 = drive(s64, x, S.xbuf, b64, P64, hier ? P.s : 1, st, ctl_of(S), &i64, false,
                                   sw > p->rel_tol ? sw : -1.0, kmin, &st1);
        if (s1 != HJ_OK && s1 != HJ_ERR_NOT_CONVERGED) return s1;
        fp64_cycles = i64.cycles;
        r0_phase1 = i64.r0_norm;
        if (st1 != hj::ST_SWITCH) {
            if (info) {
                info->outer = 0;
                info->inner_cycles = 0;
                info->fp64_cycles = fp64_cycles;
                info->rel_residual = i64.rel_residual;
                info->r0_norm = i64.r0_norm;
            }
            return s1;
        }
    }

    // phase 2: FP32 correction solves inside FP64 refinement.  Relative
    // residuals stay relative to ||f - A x_0|| for the caller's x_0, which
    // phase 1 measured if it ran.
    double rsq = 0.0;
    if ((r = fp64_residual(rsq)) != HJ_OK) return r;
    double rk_norm = std::sqrt(rsq);
    const double r0_norm = sw < 1.0 ? r0_phase1 : rk_norm;
    double rel = r0_norm > 0.0 ? rk_norm / r0_norm : 0.0;
    int64_t outer = 0, inner_cycles = 0;
    hj_status status = HJ_OK;
    while (std::isfinite(rk_norm) && rel > p->rel_tol && outer < p->max_outer) {
        hj_params Pk = P;
        Pk.rel_tol = std::max(P.rel_tol, 0.5 * p->rel_tol * r0_norm / rk_norm);
        hj_info ii{};
        const hj_status si = drive(step, e32, S.xbuf, b32, Pk, hier ? P.s : 1, st, ctl_of(S), &ii, true);
        if (si != HJ_OK && si != HJ_ERR_NOT_CONVERGED) return si;
        inner_cycles += ii.cycles;
        HJ_HIP(hj::launch_axpy_f32_to_f64(g, e32, x, st));
        ++outer;
        if ((r = fp64_residual(rsq)) != HJ_OK) return r;
        rk_norm = std::sqrt(rsq);
        if (!std::isfinite(rk_norm)) { rel = NAN; break; }
        rel = rk_norm / r0_norm;
    }
    g_err.clear();
    if (!std::isfinite(r0_norm) || !std::isfinite(rel)) status = fail(HJ_ERR_NONFINITE, "residual norm became non-finite");
    else if (rel > p->rel_tol) status = fail(HJ_ERR_NOT_CONVERGED, "max_outer reached before rel_tol");
    if (info) {
        info->outer = outer;
        info->inner_cycles = inner_cycles;
        info->fp64_cycles = fp64_cycles;
        info->rel_residual = rel;
        info->r0_norm = r0_norm;
    }
    return status;
}

// The whole 1D solve in one workgroup: cycles run in chunks of kWgChunk per
// launch (a few ms of GPU time), the solve state carried in S.ctrl.  Same stop
// rule, iterates and info as drive().
static constexpr int64_t kWgChunk = 4096;

static hj_status drive_1d_wg(const hj::Geom1 &g, int dt, const hj_params &p, const void *f, void *x, hipStream_t st,
                      DevScratch &S, hj_info *info)
{
    const int64_t maxc = p.max_cycles;
    const bool every = p.rel_tol > 0.0;
    const double tol = every ? p.rel_tol : -1.0;
    hj_status r;
    hj::Ctrl c{};
    HJ_HIP(hj::launch_ctrl_init(S.ctrl, st));
    for (int64_t cb = 0;;) {
        const int64_t ce = maxc - cb < kWgChunk ? maxc + 1 : cb + kWgChunk;
        HJ_HIP(hj::launch_solve1d_wg(dt, g, p.s, f, x, cb, ce, maxc, tol, every, S.ctrl, st));
        if (ce == maxc + 1) break;
        if (every) {
            if ((r = read_ctrl(S, st, c)) != HJ_OK) return r;
            if (c.status != hj::ST_RUNNING) break;
        }
        cb = ce;
    }
    if ((r = read_ctrl(S, st, c)) != HJ_OK) return r;
    const int64_t final_c = every && c.status != hj::ST_RUNNING ? c.done_cycle : maxc;
    if (info) {
        info->cycles = final_c;
        info->sweeps = final_c * p.s;
        info->r0_norm = std::sqrt(c.r0sq);
        info->rel_residual = c.r0sq > 0.0 ? std::sqrt(c.last_rsq) / std::sqrt(c.r0sq) : 0.0;
        if (!std::isfinite(c.last_rsq)) info->rel_residual = NAN;
    }
    if (c.status == hj::ST_NONFINITE) return fail(HJ_ERR_NONFINITE, "residual norm became non-finite");
    if (every && c.status != hj::ST_CONVERGED) return fail(HJ_ERR_NOT_CONVERGED, "max_cycles reached before rel_tol");
    return HJ_OK;
}

hj_status hj_solve_1d(int64_t n, double h, hj_dtype dtype, const void *f, void *x,
                      const hj_params *p, void *stream, hj_info *info)
{
    g_err.clear();
    if (n < 1 || n > kMaxAxis) return fail(HJ_ERR_INVALID_ARG, "n must be in [1, 2^30]");
    if (!finite_pos(h)) return fail(HJ_ERR_INVALID_ARG, "h must be finite and > 0");
    if (dtype != HJ_F64 && dtype != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    hj_status r;
    if ((r = check_ptr_dtype(f, dtype, "f", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(x, dtype, "x", false)) != HJ_OK) return r;
    if ((r = check_params(p, 1)) != HJ_OK) return r;

    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    if ((r = check_device_ptr(f, dev, "f")) != HJ_OK) return r;
    if ((r = check_device_ptr(x, dev, "x")) != HJ_OK) return r;

    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    const hj_params P = *p;
    const hj::Geom1 g = make_geom1(n, h, &P);
    const int dt = dtype == HJ_F64 ? hj::F64 : hj::F32;
    const size_t es = esize(dtype);
    const bool hier = P.method == HJ_HIERARCHICAL;
    hipStream_t st = (hipStream_t)stream;
    if (hier && !(P.flags & HJ_FLAG_LAUNCH_PER_CYCLE) && hj::solve1d_wg_supported(g, dt)) {
        if ((r = scratch_ensure(S, 0, 0)) != HJ_OK) return r;
        return drive_1d_wg(g, dt, P, f, x, st, S, info);
    }
    if (!hier && !(P.flags & HJ_FLAG_LAUNCH_PER_CYCLE)) {
        // Classical Jacobi is the cycle with one sub-iteration and no overlap
        // (Sec. 3.3: k = 1 is exactly Jacobi), so a grid that fits one
        // workgroup runs its sweeps there too, launch-free like the
        // hierarchical solve: the smallest tile that covers the grid in at
        // most 16 tiles.
        for (const int t : {64, 128, 256, 512}) {
            hj_params Q = P;
            Q.tile_x = t;
            Q.overlap_x = 0;
            Q.s = 1;
            const hj::Geom1 gq = make_geom1(n, h, &Q);
            if (!hj::solve1d_wg_supported(gq, dt)) continue;
            if ((r = scratch_ensure(S, 0, 0)) != HJ_OK) return r;
            return drive_1d_wg(gq, dt, Q, f, x, st, S, info);
        }
    }
    const int64_t nbc = hier ? hj::cycle1d_blocks(g) : hj::sweep1d_blocks(g);
    const int64_t nbr = hj::resid1d_blocks(g);
    if (nbc > INT32_MAX || nbr > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "grid too large");
    const size_t xbytes = (size_t)n * es;
    if ((r = scratch_ensure(S, 2 * xbytes, 2 * std::max(nbc, nbr))) != HJ_OK) return r;

    Step step;
    step.nb_cycle = (int)nbc;
    step.nb_resid = (int)nbr;
    step.cycle = [&](const void *xi, void *xo, bool res, double tol, const hj::Red &red) {
        return hier ? hj::launch_cycle1d(dt, g, P.s, res, f, xi, xo, red, tol, st)
                    : hj::launch_sweep1d(dt, g, res, f, xi, xo, red, tol, st);
    };
    step.resid = [&](const void *xi, double *part) {
        return hj::launch_resid1d(dt, g, f, xi, nullptr, part, st);
    };
    step.copy = [&](void *dst, const void *src) {
        return hipMemcpyAsync(dst, src, (size_t)n * es, hipMemcpyDeviceToDevice, st);
    };
    return drive(step, x, S.xbuf, xbytes, P, hier ? P.s : 1, st, ctl_of(S), info);
}

hj_status hj_residual(int32_t dim, int64_t nx, int64_t ny, int64_t ld, double hx, double hy,
                      hj_dtype dtype, const void *f, const void *x, void *r_out, double *norm2_out,
                      void *stream)
{
    g_err.clear();
    if (dim != 1 && dim != 2) return fail(HJ_ERR_INVALID_ARG, "dim must be 1 or 2");
    if (nx < 1 || nx > kMaxAxis) return fail(HJ_ERR_INVALID_ARG, "nx must be in [1, 2^30]");
    if (dim == 2 && (ny < 1 || ny > kMaxAxis)) return fail(HJ_ERR_INVALID_ARG, "ny must be in [1, 2^30]");
    if (dim == 2 && ld < nx) return fail(HJ_ERR_INVALID_ARG, "ld must be >= nx");
    if (!finite_pos(hx) || (dim == 2 && !finite_pos(hy)))
        return fail(HJ_ERR_INVALID_ARG, "spacings must be finite and > 0");
    if (dtype != HJ_F64 && dtype != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    hj_status r;
    if ((r = check_ptr_dtype(f, dtype, "f", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(x, dtype, "x", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(r_out, dtype, "r_out", true)) != HJ_OK) return r;

    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    if ((r = check_device_ptr(f, dev, "f")) != HJ_OK) return r;
    if ((r = check_device_ptr(x, dev, "x")) != HJ_OK) return r;
    if ((r = check_device_ptr(r_out, dev, "r_out")) != HJ_OK) return r;

    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    const int dt = dtype == HJ_F64 ? hj::F64 : hj::F32;
    hipStream_t st = (hipStream_t)stream;
    if (dim == 2) {
        hj_params P;
        hj_params_default(&P);
        const hj::Geom2 g = make_geom2(nx, ny, ld, hx, hy, P);
        const int64_t nb = hj::resid2d_blocks(g);
        if (nb > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "grid too large");
        if ((r = scratch_ensure(S, 0, 2 * nb)) != HJ_OK) return r;
        HJ_HIP(hj::launch_ctrl_init(S.ctrl, st));
        HJ_HIP(hj::launch_resid2d(dt, g, f, x, r_out, S.partials, st));
        HJ_HIP(hj::launch_judge(S.partials, (int)nb, S.ctrl, 0, -1.0, st));
    } else {
        const hj::Geom1 g = make_geom1(nx, hx, nullptr);
        const int64_t nb = hj::resid1d_blocks(g);
        if (nb > INT32_MAX) return fail(HJ_ERR_UNSUPPORTED, "grid too large");
        if ((r = scratch_ensure(S, 0, 2 * nb)) != HJ_OK) return r;
        HJ_HIP(hj::launch_ctrl_init(S.ctrl, st));
        HJ_HIP(hj::launch_resid1d(dt, g, f, x, r_out, S.partials, st));
        HJ_HIP(hj::launch_judge(S.partials, (int)nb, S.ctrl, 0, -1.0, st));
    }
    HJ_HIP(hipMemcpyAsync(&S.host[0], S.ctrl, sizeof(hj::Ctrl), hipMemcpyDeviceToHost, st));
    HJ_HIP(hipStreamSynchronize(st));
    if (norm2_out) *norm2_out = std::sqrt(S.host[0].last_rsq);
    if (!std::isfinite(S.host[0].last_rsq)) return fail(HJ_ERR_NONFINITE, "residual norm is non-finite");
    return HJ_OK;
}

hj_status hj_autotune(int32_t dim, int64_t nx, int64_t ny, hj_dtype dtype, void *stream,
                      hj_params *best, double *us_per_sweep)
{
    g_err.clear();
    if (dim != 1 && dim != 2) return fail(HJ_ERR_INVALID_ARG, "dim must be 1 or 2");
    if (nx < 1 || nx > kMaxAxis || (dim == 2 && (ny < 1 || ny > kMaxAxis)))
        return fail(HJ_ERR_INVALID_ARG, "nx, ny must be in [1, 2^30]");
    if (dtype != HJ_F64 && dtype != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    if (!best) return fail(HJ_ERR_INVALID_ARG, "best is NULL");
    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    hj_params P;
    double us = 0.0;
    const hj_status r = autotune_locked(dim, nx, dim == 2 ? ny : 1, dtype, 1 << 30, 1 << 30,
                                        (hipStream_t)stream, dev, S, P, us);
    if (r != HJ_OK) return r;
    *best = P;
    if (us_per_sweep) *us_per_sweep = us;
    return HJ_OK;
}

hj_status hj_autotune_solve(int64_t nx, int64_t ny, int64_t ld, double hx, double hy, hj_dtype dtype,
                            const void *f, const void *x0, const hj_tune_params *tp, void *stream,
                            hj_params *best, double *best_ms)
{
    g_err.clear();
    if (!tp || !best) return fail(HJ_ERR_INVALID_ARG, "tune params and best must not be NULL");
    if (!(tp->trial_tol > 0.0) || !std::isfinite(tp->trial_tol))
        return fail(HJ_ERR_INVALID_ARG, "trial_tol must be finite and > 0");
    if (tp->max_trial_cycles < 1) return fail(HJ_ERR_INVALID_ARG, "max_trial_cycles must be >= 1");
    if (tp->flags != 0) return fail(HJ_ERR_INVALID_ARG, "tune flags must be 0");
    if (tp->nrhs < 0 || tp->nrhs > 1024) return fail(HJ_ERR_INVALID_ARG, "nrhs must be in [0, 1024]");
    const int nrhs = tp->nrhs > 1 ? tp->nrhs : 1;
    if ((tp->tile_x == 0) != (tp->tile_y == 0)) return fail(HJ_ERR_INVALID_ARG, "give both tile extents or neither");
    if (tp->tile_x && !hj::cycle2d_supported(tp->tile_x, tp->tile_y))
        return fail(HJ_ERR_UNSUPPORTED, "unsupported 2D tile shape");
    hj_params base;
    hj_params_default(&base);
    base.rel_tol = tp->trial_tol;
    base.max_cycles = tp->max_trial_cycles;
    hj_status r;
    if ((r = check_solve_2d(nx, ny, ld, hx, hy, dtype, f, x0, &base)) != HJ_OK) return r;
    if (nrhs > 1 && (tp->rhs_stride < 0 || tp->rhs_stride / ld < ny))  // rhs_stride >= ny * ld, no overflow
        return fail(HJ_ERR_INVALID_ARG, "rhs_stride must be >= ny * ld when nrhs > 1");
    const size_t es0 = esize(dtype);
    auto rhs = [&](int k) { return (const void *)((const char *)f + (size_t)k * (size_t)tp->rhs_stride * es0); };
    for (int k = 1; k < nrhs; ++k)
        if ((r = check_solve_2d(nx, ny, ld, hx, hy, dtype, rhs(k), x0, &base)) != HJ_OK) return r;

    // candidates: exact regime first (they reveal the classical sweep count),
    // then overlaps a little short of it (owned points a few points inside
    // the stale halo's reach, where its influence is small and the count
    // often stays that of the exact regime at less redundant loading), then
    // small overlaps
    std::vector<hj_params> cands;
    const int tiles[][2] = {{64, 128}, {64, 64}, {32, 64}, {64, 32}, {32, 32}};
    for (const bool exact : {true, false}) {
        for (auto &t : tiles) {
            const int tx = tp->tile_x ? tp->tile_x : t[0], ty = tp->tile_y ? tp->tile_y : t[1];
            if (tp->tile_x && (t[0] != tiles[0][0] || t[1] != tiles[0][1])) continue;  // the given tile once
            for (const int s : {32, 24, 16, 12, 8, 4}) {
                const int three_halves = (3 * s / 2 + 1) & ~1;
                for (const int o : {2 * s - 2, 2 * s - 6, 2 * s - 10, three_halves, s + 6, s + 2, 8, 4, 2, 0}) {
                    if ((o == 2 * s - 2) != exact || o >= std::min(tx, ty) || o < 0) continue;
                    if (!exact && o >= 2 * s - 2) continue;
                    if (load_factor(nx, ny, tx, ty, o, o) > kMaxLoadFactor) continue;
                    hj_params P = base;
                    P.tile_x = tx;
                    P.tile_y = ty;
                    P.s = s;
                    P.overlap_x = P.overlap_y = o;
                    if (!hj::cycle2d_runnable(make_geom2(nx, ny, ld, hx, hy, P))) continue;
                    bool dup = false;
                    for (const hj_params &c : cands)
                        dup = dup || (c.tile_x == P.tile_x && c.tile_y == P.tile_y && c.s == P.s &&
                                      c.overlap_x == P.overlap_x);
                    if (!dup) cands.push_back(P);
                }
            }
        }
    }
    if (cands.empty()) return fail(HJ_ERR_UNSUPPORTED, "autotune_solve: no candidate tile fits the grid");
    int64_t npart = 0;
    for (const hj_params &P : cands) {
        int64_t np = 0;
        if ((r = solve_2d_partials(nx, ny, ld, hx, hy, P, np)) != HJ_OK) return r;
        npart = std::max(npart, np);
    }
    int dev = 0;
    if ((r = solve_device(f, x0, dev)) != HJ_OK) return r;
    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    const size_t es = esize(dtype);
    const size_t xbytes = (size_t)ny * (size_t)ld * es;
    // the trial iterate, then the solve's two spare arrays
    if ((r = scratch_ensure(S, 3 * xbytes, npart)) != HJ_OK) return r;
    if (!S.tev[0]) {
        HJ_HIP(hipEventCreate(&S.tev[0]));
        HJ_HIP(hipEventCreate(&S.tev[1]));
    }
    hipStream_t st = (hipStream_t)stream;
    void *xw = S.xbuf;
    void *xs = (char *)S.xbuf + xbytes;
    const int dt = dtype == HJ_F64 ? hj::F64 : hj::F32;
    HJ_HIP(hipMemsetAsync(xs, 0, 2 * xbytes, st));  // the per-cycle timings run on zeros
    auto restore = [&]() {
        return hipMemcpy2DAsync(xw, (size_t)ld * es, x0, (size_t)ld * es, (size_t)nx * es, (size_t)ny,
                                hipMemcpyDeviceToDevice, st);
    };
    // time per cycle from a few fixed cycles between the spare arrays
    auto cycle_ms = [&](const hj_params &P, double &ms) -> hj_status {
        const hj::Geom2 g = make_geom2(nx, ny, ld, hx, hy, P);
        const hj::Red none{nullptr, nullptr, S.ctrl, 0, 0};
        void *a = xs, *b = (char *)xs + xbytes;
        HJ_HIP(hj::launch_cycle2d(dt, g, P.s, false, f, a, b, none, -1.0, st));
        constexpr int k = 6;
        HJ_HIP(hipEventRecord(S.tev[0], st));
        for (int i = 0; i < k; ++i) HJ_HIP(hj::launch_cycle2d(dt, g, P.s, false, f, (i & 1) ? b : a, (i & 1) ? a : b, none, -1.0, st));
        HJ_HIP(hipEventRecord(S.tev[1], st));
        HJ_HIP(hipEventSynchronize(S.tev[1]));
        float e = 0.0f;
        HJ_HIP(hipEventElapsedTime(&e, S.tev[0], S.tev[1]));
        ms = (double)e / k;
        return HJ_OK;
    };
    double best_t = INFINITY;
    // per right-hand side, a lower bound on its classical sweep count to trial_tol
    std::vector<int64_t> n_classical((size_t)nrhs, 0);
    hj_params winner = cands[0];
    for (const hj_params &P0 : cands) {
        double tc = 0.0;
        if ((r = cycle_ms(P0, tc)) != HJ_OK) return r;
        const bool exact = P0.overlap_x >= 2 * P0.s - 2;
        bool known = true;
        double floor_t = 0.0;
        for (const int64_t nc : n_classical) {
            known = known && nc > 0;
            floor_t += tc * (double)((nc + P0.s - 1) / P0.s);
        }
        if (known && floor_t >= best_t) continue;
        double total = 0.0;
        bool ok = true;
        for (int k = 0; k < nrhs && ok; ++k) {
            hj_params P = P0;
            if (std::isfinite(best_t))
                P.max_cycles = std::max<int64_t>(
                    1, std::min<int64_t>(P.max_cycles, (int64_t)((best_t - total) / tc) + 2));
            HJ_HIP(restore());
            hj_info info{};
            HJ_HIP(hipEventRecord(S.tev[0], st));
            const hj_status sr = solve_2d_on(nx, ny, ld, hx, hy, dtype, rhs(k), xw, P, st, xs, ctl_of(S), &info);
            HJ_HIP(hipEventRecord(S.tev[1], st));
            HJ_HIP(hipEventSynchronize(S.tev[1]));
            if (sr == HJ_ERR_HIP || sr == HJ_ERR_INVALID_ARG) return sr;
            if (sr != HJ_OK) {
                ok = false;
                break;
            }
            float e = 0.0f;
            HJ_HIP(hipEventElapsedTime(&e, S.tev[0], S.tev[1]));
            if (exact && info.cycles > 0) {
                // an exact-regime cycle is s classical sweeps: more than
                // (cycles - 1) s sweeps were needed
                n_classical[(size_t)k] = std::max<int64_t>(n_classical[(size_t)k], (info.cycles - 1) * P.s + 1);
            }
            total += (double)e;
            if (total >= best_t) ok = false;  // lost already
        }
        if (ok && total < best_t) {
            best_t = total;
            winner = P0;
        }
    }
    g_err.clear();
    if (!std::isfinite(best_t))
        return fail(HJ_ERR_NOT_CONVERGED, "autotune_solve: no candidate reached trial_tol on every right-hand side");
    *best = winner;
    best->max_cycles = tp->max_trial_cycles;
    if (best_ms) *best_ms = best_t;
    return HJ_OK;
}

hj_status hj_autotune_batch(const hj_problem *probs, int64_t nprob, hj_dtype dtype, void *stream,
                            hj_params *p2, hj_params *p1)
{
    g_err.clear();
    if (!probs) return fail(HJ_ERR_INVALID_ARG, "probs is NULL");
    if (nprob < 1 || nprob > (1 << 24)) return fail(HJ_ERR_INVALID_ARG, "nprob must be in [1, 2^24]");
    if (dtype != HJ_F64 && dtype != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    hj_status r;
    for (int64_t i = 0; i < nprob; ++i)
        if ((r = check_problem(probs[i], dtype, -1, i)) != HJ_OK) return r;
    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    hj_params P2, P1;
    hj_params_default(&P2);
    hj_params_default(&P1);
    if ((r = tune_batch_locked(probs, nprob, dtype, (hipStream_t)stream, dev, S, P2, P1)) != HJ_OK) return r;
    if (p2) *p2 = P2;
    if (p1) *p1 = P1;
    return HJ_OK;
}

// HJ_BATCH_WG1D: workgroup i runs problem i's whole solve (the one-workgroup
// body of hj_solve_1d); cycles in launches of kWgChunk, the per-problem
// states read back between launches in tolerance mode.  Called with the
// device's scratch lock held, problems already checked.
static hj_status solve_batched_wg1d(const hj_problem *probs, int64_t nprob, const hj_batch_params &p, hj_dtype dtype,
                             hipStream_t st, BatchScratch &B, hj_info *infos)
{
    const hj_params &P1 = p.p1;
    const int dt = dtype == HJ_F64 ? hj::F64 : hj::F32;
    std::vector<hj::WgProb> table((size_t)nprob);
    int64_t max_n = 0, max_nt = 0;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj_problem &q = probs[i];
        if (q.dim != 1) return fail(HJ_ERR_UNSUPPORTED, "HJ_BATCH_WG1D takes 1D problems only");
        const hj::Geom1 g = make_geom1(q.nx, q.hx, &P1);
        if (!hj::solve1d_wg_supported(g, dt))
            return fail(HJ_ERR_UNSUPPORTED, "problem " + std::to_string(i) +
                                                ": HJ_BATCH_WG1D needs tiles of 64..512 points, at most 16 tiles "
                                                "and 3 n element sizes within the workgroup's LDS (150 KiB on gfx950)");
        table[(size_t)i] = hj::WgProb{g, q.f, q.x};
        max_n = std::max(max_n, g.n);
        max_nt = std::max(max_nt, g.nt);
    }
    const size_t tbytes = ((size_t)nprob * sizeof(hj::WgProb) + 255) / 256 * 256;
    const size_t need = tbytes + (size_t)nprob * sizeof(hj::Ctrl);
    if (need > B.wg_bytes) {
        if (B.wg) HJ_HIP(hipFree(B.wg));
        B.wg = nullptr;
        B.wg_bytes = 0;
        HJ_HIP(hipMalloc(&B.wg, need));
        B.wg_bytes = need;
    }
    hj::WgProb *dprobs = (hj::WgProb *)B.wg;
    hj::Ctrl *ctrls = (hj::Ctrl *)((char *)B.wg + tbytes);
    HJ_HIP(hipMemcpyAsync(dprobs, table.data(), (size_t)nprob * sizeof(hj::WgProb), hipMemcpyHostToDevice, st));
    HJ_HIP(hj::launch_ctrl_init_n(ctrls, nprob, st));

    const int64_t maxc = p.max_cycles;
    const bool every = p.rel_tol > 0.0;
    const double tol = every ? p.rel_tol : -1.0;
    std::vector<hj::Ctrl> hc((size_t)nprob);
    auto read_back = [&]() -> hj_status {
        HJ_HIP(hipMemcpyAsync(hc.data(), ctrls, (size_t)nprob * sizeof(hj::Ctrl), hipMemcpyDeviceToHost, st));
        HJ_HIP(hipStreamSynchronize(st));
        return HJ_OK;
    };
    hj_status r;
    for (int64_t cb = 0;;) {
        const int64_t ce = maxc - cb < kWgChunk ? maxc + 1 : cb + kWgChunk;
        HJ_HIP(hj::launch_solve1d_wg_batch(dt, P1.tile_x, dprobs, nprob, max_n, max_nt, P1.s, cb, ce, maxc, tol,
                                           every, ctrls, st));
        if (ce == maxc + 1) break;
        if (every) {
            if ((r = read_back()) != HJ_OK) return r;
            if (std::none_of(hc.begin(), hc.end(), [](const hj::Ctrl &c) { return c.status == hj::ST_RUNNING; }))
                break;
        }
        cb = ce;
    }
    if ((r = read_back()) != HJ_OK) return r;

    hj_status status = HJ_OK;
    int64_t bad = -1;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj::Ctrl &c = hc[(size_t)i];
        const int64_t used = every && c.status != hj::ST_RUNNING ? c.done_cycle : maxc;
        if (infos) {
            infos[i].cycles = used;
            infos[i].sweeps = used * P1.s;
            infos[i].r0_norm = std::sqrt(c.r0sq);
            infos[i].rel_residual = c.r0sq > 0.0 ? std::sqrt(c.last_rsq) / std::sqrt(c.r0sq) : 0.0;
            if (!std::isfinite(c.last_rsq)) infos[i].rel_residual = NAN;
        }
        if (c.status == hj::ST_NONFINITE) {
            status = HJ_ERR_NONFINITE;
            bad = i;
        } else if (c.status != hj::ST_CONVERGED && every && status == HJ_OK) {
            status = HJ_ERR_NOT_CONVERGED;
            bad = i;
        }
    }
    if (status == HJ_ERR_NONFINITE)
        return fail(status, "problem " + std::to_string(bad) + ": residual norm became non-finite");
    if (status == HJ_ERR_NOT_CONVERGED)
        return fail(status, "problem " + std::to_string(bad) + " did not reach rel_tol within max_cycles");
    return HJ_OK;
}

hj_status hj_solve_batched(const hj_problem *probs, int64_t nprob, const hj_batch_params *p,
                           void *stream, hj_info *infos)
{
    g_err.clear();
    if (!probs) return fail(HJ_ERR_INVALID_ARG, "probs is NULL");
    if (nprob < 1 || nprob > (1 << 24)) return fail(HJ_ERR_INVALID_ARG, "nprob must be in [1, 2^24]");
    if (!p) return fail(HJ_ERR_INVALID_ARG, "params is NULL");
    const hj_dtype dt = (hj_dtype)p->dtype;
    if (dt != HJ_F64 && dt != HJ_F32) return fail(HJ_ERR_INVALID_ARG, "unknown dtype");
    if (std::isnan(p->rel_tol)) return fail(HJ_ERR_INVALID_ARG, "rel_tol is NaN");
    if (p->max_cycles < 1) return fail(HJ_ERR_INVALID_ARG, "max_cycles must be >= 1");
    if (p->graph_cycles < 0 || p->graph_cycles > 1024)
        return fail(HJ_ERR_INVALID_ARG, "graph_cycles must be in [0, 1024]");
    if (p->flags & ~(HJ_BATCH_AUTOTUNE | HJ_BATCH_REFINE | HJ_BATCH_WG1D))
        return fail(HJ_ERR_INVALID_ARG, "unknown bits in flags");
    const bool tune = (p->flags & HJ_BATCH_AUTOTUNE) != 0;
    const bool refine = (p->flags & HJ_BATCH_REFINE) != 0;
    const bool wg1d = (p->flags & HJ_BATCH_WG1D) != 0;
    if (wg1d && (tune || refine))
        return fail(HJ_ERR_UNSUPPORTED, "HJ_BATCH_WG1D does not combine with HJ_BATCH_AUTOTUNE or HJ_BATCH_REFINE");
    if (refine && dt != HJ_F64) return fail(HJ_ERR_INVALID_ARG, "refined batches take FP64 problems");
    if (refine && !(p->rel_tol > 0.0)) return fail(HJ_ERR_INVALID_ARG, "refined batches need rel_tol > 0");
    if (p->max_outer < 0) return fail(HJ_ERR_INVALID_ARG, "max_outer must be >= 0");
    hj_status r;
    int64_t n2 = 0, n1 = 0, min_nx = INT64_MAX, min_ny = INT64_MAX;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj_problem &q = probs[i];
        if ((r = check_problem(q, dt, -1, i)) != HJ_OK) return r;
        if (q.dim == 2) {
            ++n2;
            min_nx = std::min(min_nx, q.nx);
            min_ny = std::min(min_ny, q.ny);
        } else {
            ++n1;
        }
    }
    if (!tune) {
        if (n2) {
            if ((r = check_params(&p->p2, 2)) != HJ_OK) return r;
            if (p->p2.method != HJ_HIERARCHICAL || p->p2.flags != 0)
                return fail(HJ_ERR_UNSUPPORTED, "batched 2D cycles are hierarchical, register-resident");
            if (!hj::batch2d_supported(p->p2.tile_x, p->p2.tile_y))
                return fail(HJ_ERR_UNSUPPORTED, "batched 2D tiles: tile_x in {32, 64}, tile_y in {16, 32, 64, 128}");
            if (min_nx < p->p2.tile_x || min_ny < p->p2.tile_y)
                return fail(HJ_ERR_UNSUPPORTED, "every 2D problem of a batch needs nx >= tile_x and ny >= tile_y");
        }
        if (n1) {
            if ((r = check_params(&p->p1, 1)) != HJ_OK) return r;
            if (p->p1.method != HJ_HIERARCHICAL)
                return fail(HJ_ERR_UNSUPPORTED, "batched 1D cycles are hierarchical");
        }
    }

    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    for (int64_t i = 0; i < nprob; ++i)
        if ((r = check_problem(probs[i], dt, dev, i)) != HJ_OK) return r;

    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    hipStream_t st = (hipStream_t)stream;
    if (wg1d) return solve_batched_wg1d(probs, nprob, *p, dt, st, g_bat[dev], infos);
    hj_params P2 = p->p2, P1 = p->p1;
    if (tune && (r = tune_batch_locked(probs, nprob, dt, st, dev, S, P2, P1)) != HJ_OK) return r;
    BatchScratch &B = g_bat[dev];
    const double tol = p->rel_tol > 0.0 ? p->rel_tol : -1.0;
    hj::BRefine rf{};
    if (refine) {
        rf.refine = 1;
        rf.max_outer = p->max_outer > 0 ? p->max_outer : 8;
        rf.switch_tol = std::min(1.0, 1e4 * tol);
        rf.inner_min = 1e-6;
        rf.fmax = 1.0 / 80.0;  // FP32 then takes at least one decade (tol / 8F >= 10 tol)
    }
    if ((r = run_batch(probs, nprob, dt, tol, p->max_cycles, rf, P2, P1, p->graph_cycles ? p->graph_cycles : 8,
                       st, S, B)) != HJ_OK)
        return r;

    hj_status status = HJ_OK;
    int64_t bad = -1;
    for (int64_t i = 0; i < nprob; ++i) {
        const hj::BState &c = B.host[i];
        const int s_dim = probs[i].dim == 2 ? P2.s : P1.s;
        if (infos) {
            infos[i].cycles = c.used;
            infos[i].sweeps = c.used * s_dim;
            infos[i].r0_norm = std::sqrt(c.r0sq);
            infos[i].rel_residual = c.r0sq > 0.0 ? std::sqrt(c.rsq) / std::sqrt(c.r0sq) : 0.0;
            if (!std::isfinite(c.rsq)) infos[i].rel_residual = NAN;
        }
        if (c.status == hj::ST_NONFINITE) {
            status = HJ_ERR_NONFINITE;
            bad = i;
        } else if (c.status != hj::ST_CONVERGED && tol > 0.0 && status == HJ_OK) {
            status = HJ_ERR_NOT_CONVERGED;
            bad = i;
        }
    }
    if (status == HJ_ERR_NONFINITE)
        return fail(status, "problem " + std::to_string(bad) + ": residual norm became non-finite");
    if (status == HJ_ERR_NOT_CONVERGED)
        return fail(status, "problem " + std::to_string(bad) + " did not reach rel_tol within max_cycles");
    return HJ_OK;
}

hj_status hj_solve_vc_2d(const hj_vc_problem *prob, const double *f, double *u, const hj_params *p,
                         void *stream, hj_info *infos)
{
    g_err.clear();
    hj_status r;
    if ((r = check_vc_problem(prob)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(f, HJ_F64, "f", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(u, HJ_F64, "u", false)) != HJ_OK) return r;
    if ((r = check_params(p, 2)) != HJ_OK) return r;
    if (p->method == HJ_HIERARCHICAL && ((p->tile_x ? p->tile_x : 32) > 64 || (p->tile_y ? p->tile_y : 32) > 64))
        return fail(HJ_ERR_UNSUPPORTED, "variable-coefficient tiles are at most 64 x 64");
    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) return fail(HJ_ERR_UNSUPPORTED, "device index out of range");
    if ((r = check_device_ptr(prob->a, dev, "a")) != HJ_OK) return r;
    if ((r = check_device_ptr(f, dev, "f")) != HJ_OK) return r;
    if ((r = check_device_ptr(u, dev, "u")) != HJ_OK) return r;
    DevScratch &S = g_scr[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    if (p->method == HJ_HIERARCHICAL && prob->batch > 1)
        return solve_vc_batched(*prob, f, u, *p, (hipStream_t)stream, dev, S, infos);
    return solve_vc_locked(*prob, f, u, *p, (hipStream_t)stream, S, infos);
}

hj_status hj_vc_grad_a(const hj_vc_problem *prob, const double *u, const double *lam, double *grad,
                       int64_t ld_grad, void *stream)
{
    g_err.clear();
    hj_status r;
    if ((r = check_vc_problem(prob)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(u, HJ_F64, "u", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(lam, HJ_F64, "lam", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(grad, HJ_F64, "grad", false)) != HJ_OK) return r;
    if (ld_grad < prob->nx + 2) return fail(HJ_ERR_INVALID_ARG, "ld_grad must be >= nx + 2");
    int dev = 0;
    HJ_HIP(hipGetDevice(&dev));
    if ((r = check_device_ptr(u, dev, "u")) != HJ_OK) return r;
    if ((r = check_device_ptr(lam, dev, "lam")) != HJ_OK) return r;
    if ((r = check_device_ptr(grad, dev, "grad")) != HJ_OK) return r;
    if ((r = check_device_ptr(prob->a, dev, "a")) != HJ_OK) return r;
    hj_params P;
    hj_params_default(&P);
    const hj::GeomVC g = make_geom_vc(*prob, P);
    hipStream_t st = (hipStream_t)stream;
    HJ_HIP(hj::launch_grad_a_vc(g, u, lam, prob->batch, prob->batch_stride, grad, ld_grad, st));
    HJ_HIP(hipStreamSynchronize(st));
    return HJ_OK;
}

hj_status hj_solve_adjoint(const hj_adjoint_desc *d, void *stream, hj_info *infos)
{
    g_err.clear();
    if (!d) return fail(HJ_ERR_INVALID_ARG, "descriptor is NULL");
    // everything the gradient step needs is checked before the solve runs
    hj_status r;
    if ((r = check_vc_problem(&d->prob)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(d->dl_du, HJ_F64, "dl_du", false)) != HJ_OK) return r;
    if ((r = check_ptr_dtype(d->lam, HJ_F64, "lam", false)) != HJ_OK) return r;
    if (d->dl_da) {
        if (!d->u) return fail(HJ_ERR_INVALID_ARG, "u is NULL while dl_da is requested");
        if ((r = check_ptr_dtype(d->u, HJ_F64, "u", false)) != HJ_OK) return r;
        if ((r = check_ptr_dtype(d->dl_da, HJ_F64, "dl_da", false)) != HJ_OK) return r;
        if (d->ld_grad < d->prob.nx + 2) return fail(HJ_ERR_INVALID_ARG, "ld_grad must be >= nx + 2");
        int dev = 0;
        HJ_HIP(hipGetDevice(&dev));
        if ((r = check_device_ptr(d->u, dev, "u")) != HJ_OK) return r;
        if ((r = check_device_ptr(d->dl_da, dev, "dl_da")) != HJ_OK) return r;
    }
    r = hj_solve_vc_2d(&d->prob, d->dl_du, d->lam, &d->params, stream, infos);
    if (r != HJ_OK) return r;
    if (d->dl_da) return hj_vc_grad_a(&d->prob, d->u, d->lam, d->dl_da, d->ld_grad, stream);
    return HJ_OK;
}

int64_t hj_axis_tiles(int64_t n, int32_t tile, int32_t overlap)
{
    if (n < 1 || n > kMaxAxis || tile < 1 || overlap < 0 || overlap >= tile) return -1;
    return hj::axis_count((int)n, tile, overlap);
}

const char *hj_status_string(hj_status s)
{
    switch (s) {
    case HJ_OK: return "HJ_OK";
    case HJ_ERR_INVALID_ARG: return "HJ_ERR_INVALID_ARG";
    case HJ_ERR_NOT_CONVERGED: return "HJ_ERR_NOT_CONVERGED";
    case HJ_ERR_NONFINITE: return "HJ_ERR_NONFINITE";
    case HJ_ERR_UNSUPPORTED: return "HJ_ERR_UNSUPPORTED";
    case HJ_ERR_HIP: return "HJ_ERR_HIP";
    default: break;
    }
    return "HJ_ERR_UNKNOWN";
}

const char *hj_last_error(void) { return g_err.c_str(); }

const char *hj_version(void) { return "hj 0.1 (gfx950)"; }

}  // extern "C"
