// hj_solve1d_wg.hip -- a whole 1D hierarchical solve inside one workgroup.
//
// When every tile of a 1D problem fits in one workgroup (at most 16 register
// tiles, one per wavefront) and the grid fits in LDS, a cycle needs no kernel
// launch of its own.  The two global iterates and f sit in LDS; each
// wavefront runs its tile's cycle in registers with the same body as the
// per-cycle kernel (load with a frozen halo, s sweeps, write-back of the owned
// points: Sec. 3.3, with the overlap of Sec. 3.5); the workgroup barrier that
// ends the cycle is the global synchronisation between cycles.  The residual
// of the iterate a cycle reads is reduced in the same pass and judged at once,
// so the solve stops at the same iterate as the per-cycle path, and the
// iterates agree with it bit for bit.  At the paper's 1D size (256 points) a
// cycle then costs about a microsecond instead of a launch.
#include <algorithm>

#include "hj_launch.h"
#include "hj_tiles.h"

namespace hj {
namespace {

constexpr int kWgThreads = 1024;              // launch bound; a launch has one wavefront per tile
constexpr int kWgMaxTiles = kWgThreads / 64;  // 16
constexpr size_t kWgLdsCap = 150 * 1024;      // f and the two iterates, at most
constexpr size_t kWgLdsDefault = 60 * 1024;   // without the device's opt-in limit

// LDS a workgroup may take for f and the iterates on the current device: the
// opt-in limit per workgroup (160 KiB on gfx950) less the static arrays,
// capped at kWgLdsCap; 60 KiB if the device does not report it.
size_t wg_max_lds()
{
    static size_t cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return kWgLdsDefault;
    if (!cache[dev]) {
        int v = 0;
        size_t lim = kWgLdsDefault;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess &&
            v > 2048)
            lim = std::min(kWgLdsCap, std::max(kWgLdsDefault, (size_t)v - 1024));
        cache[dev] = lim;
    }
    return cache[dev];
}

// Dynamic LDS above the default 64 KiB needs the kernel's opt-in.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds)
{
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// v from lane CTRL selects, 0 in rows ROW_MASK leaves out.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_or_zero(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), in every lane:
// quads, half rows and rows of 16 by lane permutations, then rows 0+1 and
// 2+3 by broadcasts of lane 15 of a row into the next, and the total in lane
// 63 read back as a uniform value.
__device__ __forceinline__ double wave_total(double v)
{
    v += dpp_or_zero<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_or_zero<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_or_zero<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_or_zero<0x140, 0xf>(v);  // row_mirror
    v += dpp_or_zero<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_or_zero<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Cycles [c_begin, c_end) of one solve by the calling workgroup (one
// wavefront per tile); c_end <= maxc + 1.  The pass for c == maxc runs no
// sweep (it only evaluates the residual of iterate maxc).  x holds iterate
// c_begin on entry and, on return, the iterate the solve stopped at
// (tolerance mode) or iterate c_end (c_end <= maxc) / maxc.  every: judge
// every iterate (tolerance mode), else only iterates 0 and maxc.  A solve
// that has stopped returns at once.
template <typename T, int TT>
__device__ __forceinline__ void solve_body(const Geom1 &g, const T *__restrict__ f, T *__restrict__ x, int s,
                                           int64_t c_begin, int64_t c_end, int64_t maxc, double tol, int every,
                                           Ctrl *ctrl, T *smem, double (&red)[2][kWgThreads / 64])
{
    // Solve state, identical in every thread (read before any thread of this
    // launch writes the block: the writes below follow at least one barrier).
    int32_t status = ctrl->status;
    if (every && status != ST_RUNNING) return;
    double r0sq = ctrl->r0sq, last = ctrl->last_rsq;
    int64_t done = ctrl->done_cycle;

    const int n = (int)g.n;
    const int nth = (int)blockDim.x;
    T *fl = smem;
    T *b0 = fl + n;
    T *b1 = b0 + n;
    for (int i = (int)threadIdx.x; i < n; i += nth) {
        fl[i] = f[i];
        b0[i] = x[i];
    }
    // slots of wavefronts the workgroup does not have stay 0
    for (int w = (int)threadIdx.x; w < 2 * kWgMaxTiles; w += nth) red[w / kWgMaxTiles][w % kWgMaxTiles] = 0.0;
    __syncthreads();

    int64_t c = c_begin;
    bool stop = false;
    for (; c < c_end; ++c) {
        const bool odd = ((c - c_begin) & 1) != 0;
        const T *xin = odd ? b1 : b0;
        T *xout = odd ? b0 : b1;
        const double mine = reg_tiles_1d<T, TT, true>(g, 0, fl, xin, xout, c < maxc ? s : 0);
        const double wsum = wave_total(mine);
        if ((threadIdx.x & 63) == 0) red[odd][threadIdx.x >> 6] = wsum;
        // The one barrier of a cycle: every write-back (and wavefront sum) of
        // this cycle is visible after it, and every read of xin is done before
        // the next cycle overwrites it.  red alternates with the cycle parity,
        // so the next cycle's sums land in the other half while slow
        // wavefronts still read this one.
        __syncthreads();
        double p[kWgMaxTiles];
#pragma unroll
        for (int w = 0; w < kWgMaxTiles; ++w) p[w] = red[odd][w];
#pragma unroll
        for (int h = kWgMaxTiles / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int w = 0; w < h; ++w) p[w] += p[w + h];
        const double tot = p[0];
        if (status == ST_RUNNING && (every || c == 0 || c == maxc)) {
            if (c == 0) r0sq = tot;
            last = tot;
            // Exact verdict rel = sqrt(tot) / sqrt(r0sq) <= tol, skipped while
            // tot exceeds tol^2 r0sq by a margin (1e-6) far above the rounding
            // of either form: then rel > tol for certain.  Only a normal bound
            // is trusted (no underflow).
            const double bound = tol * tol * r0sq * (1.0 + 1e-6);
            if (!isfinite(tot)) status = ST_NONFINITE;
            else if (!(bound >= 0x1p-1000 && bound <= 0x1p1000 && tot > bound)) {
                const double rel = r0sq > 0.0 ? sqrt(tot) / sqrt(r0sq) : 0.0;
                if (rel <= tol) status = ST_CONVERGED;
            }
            if (status != ST_RUNNING) done = c;
        }
        if (every && status != ST_RUNNING) {
            stop = true;
            break;
        }
    }
    // Iterate k sits in buffer (k - c_begin) & 1; after the pass for maxc
    // both buffers hold iterate maxc.
    const int64_t k = stop ? c : c_end;
    const T *res = ((k - c_begin) & 1) ? b1 : b0;
    for (int i = (int)threadIdx.x; i < n; i += nth) x[i] = res[i];
    if (threadIdx.x == 0) {
        ctrl->r0sq = r0sq;
        ctrl->last_rsq = last;
        ctrl->iter = k;
        ctrl->done_cycle = done;
        ctrl->status = status;
    }
}

// One solve; launched with 64 g.nt threads.
template <typename T, int TT>
__global__ __launch_bounds__(kWgThreads) void k_solve1d_wg(Geom1 g, const T *__restrict__ f, T *__restrict__ x,
                                                           int s, int64_t c_begin, int64_t c_end, int64_t maxc,
                                                           double tol, int every, Ctrl *ctrl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2][kWgThreads / 64];  // wavefront sums, by cycle parity
    solve_body<T, TT>(g, f, x, s, c_begin, c_end, maxc, tol, every, ctrl, (T *)smem, red);
}

// Workgroup b solves problem b of a batch; launched with 64 max(nt) threads.
template <typename T, int TT>
__global__ __launch_bounds__(kWgThreads) void k_solve1d_wg_batch(const WgProb *__restrict__ probs, int s,
                                                                 int64_t c_begin, int64_t c_end, int64_t maxc,
                                                                 double tol, int every, Ctrl *ctrls)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2][kWgThreads / 64];
    const WgProb q = probs[blockIdx.x];
    solve_body<T, TT>(q.g, (const T *)q.f, (T *)q.x, s, c_begin, c_end, maxc, tol, every, ctrls + blockIdx.x,
                      (T *)smem, red);
}

__global__ void k_ctrl_init_n(Ctrl *ctrls, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Ctrl c;
    c.r0sq = 0.0;
    c.last_rsq = 0.0;
    c.iter = 0;
    c.done_cycle = -1;
    c.stop_at = INT64_MAX;
    c.status = ST_RUNNING;
    c.pad = 0;
    c.sw_tol = -1.0;
    c.sw_min_c = 0;
    ctrls[i] = c;
}

template <typename T>
hipError_t launch_t(const Geom1 &g, int s, const void *f, void *x, int64_t c_begin, int64_t c_end, int64_t maxc,
                    double tol, bool every, Ctrl *ctrl, hipStream_t st)
{
    const size_t lds = 3 * (size_t)g.n * sizeof(T);
    const int ev = every ? 1 : 0;
    const unsigned nth = 64u * (unsigned)g.nt;  // one wavefront per tile
#define HJ_WG(TT)                                                                                            \
    case TT:                                                                                                 \
        if (hipError_t e = allow_lds(k_solve1d_wg<T, TT>, lds); e != hipSuccess) return e;                   \
        k_solve1d_wg<T, TT><<<1, nth, lds, st>>>(g, (const T *)f, (T *)x, s, c_begin, c_end, maxc, tol, ev, \
                                                 ctrl);                                                      \
        break;
    switch (g.t) {
        HJ_WG(64)
        HJ_WG(128)
        HJ_WG(256)
        HJ_WG(512)
    default:
        return hipErrorInvalidValue;
    }
#undef HJ_WG
    return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_t(int tt, const WgProb *probs, int64_t nprob, int64_t max_n, int64_t max_nt, int s,
                          int64_t c_begin, int64_t c_end, int64_t maxc, double tol, bool every, Ctrl *ctrls,
                          hipStream_t st)
{
    const size_t lds = 3 * (size_t)max_n * sizeof(T);
    const int ev = every ? 1 : 0;
    const unsigned nth = 64u * (unsigned)max_nt;
    const unsigned nb = (unsigned)nprob;
#define HJ_WG(TT)                                                                                               \
    case TT:                                                                                                    \
        if (hipError_t e = allow_lds(k_solve1d_wg_batch<T, TT>, lds); e != hipSuccess) return e;               \
        k_solve1d_wg_batch<T, TT><<<nb, nth, lds, st>>>(probs, s, c_begin, c_end, maxc, tol, ev, ctrls);       \
        break;
    switch (tt) {
        HJ_WG(64)
        HJ_WG(128)
        HJ_WG(256)
        HJ_WG(512)
    default:
        return hipErrorInvalidValue;
    }
#undef HJ_WG
    return hipGetLastError();
}

}  // namespace

bool solve1d_wg_supported(const Geom1 &g, int dt)
{
    const size_t es = dt == F64 ? sizeof(double) : sizeof(float);
    const bool tile = g.t == 64 || g.t == 128 || g.t == 256 || g.t == 512;
    return tile && g.nt >= 1 && g.nt <= kWgMaxTiles && 3 * (size_t)g.n * es <= wg_max_lds();
}

hipError_t launch_solve1d_wg(int dt, const Geom1 &g, int s, const void *f, void *x, int64_t c_begin,
                             int64_t c_end, int64_t maxc, double tol, bool every, Ctrl *ctrl, hipStream_t st)
{
    if (!solve1d_wg_supported(g, dt) || c_begin < 0 || c_end <= c_begin || c_end - 1 > maxc || s < 1)
        return hipErrorInvalidValue;
    if (dt == F64) return launch_t<double>(g, s, f, x, c_begin, c_end, maxc, tol, every, ctrl, st);
    return launch_t<float>(g, s, f, x, c_begin, c_end, maxc, tol, every, ctrl, st);
}

hipError_t launch_solve1d_wg_batch(int dt, int tt, const WgProb *probs, int64_t nprob, int64_t max_n,
                                   int64_t max_nt, int s, int64_t c_begin, int64_t c_end, int64_t maxc, double tol,
                                   bool every, Ctrl *ctrls, hipStream_t st)
{
    const size_t es = dt == F64 ? sizeof(double) : sizeof(float);
    if (nprob < 1 || nprob > INT32_MAX || max_nt < 1 || max_nt > kWgMaxTiles || max_n < 1 ||
        3 * (size_t)max_n * es > wg_max_lds() || c_begin < 0 || c_end <= c_begin || c_end - 1 > maxc || s < 1)
        return hipErrorInvalidValue;
    if (dt == F64) return launch_batch_t<double>(tt, probs, nprob, max_n, max_nt, s, c_begin, c_end, maxc, tol, every, ctrls, st);
    return launch_batch_t<float>(tt, probs, nprob, max_n, max_nt, s, c_begin, c_end, maxc, tol, every, ctrls, st);
}

hipError_t launch_ctrl_init_n(Ctrl *ctrls, int64_t n, hipStream_t st)
{
    if (n < 1) return hipSuccess;
    k_ctrl_init_n<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(ctrls, n);
    return hipGetLastError();
}

}  // namespace hj
