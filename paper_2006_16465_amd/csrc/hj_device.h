// hj_device.h -- device-side building blocks shared by the HIP kernels:
// the control block of a solve, the tile partition, the XCD-aware block
// mapping and the deterministic grid-wide FP64 sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hj {

// Device-resident state of one solve.  The residual of the iterate a cycle
// kernel reads is reduced inside that kernel; its last workgroup to finish
// updates this block, so the host only polls it now and then.
struct Ctrl {
    double r0sq;         // ||r_0||^2
    double last_rsq;     // ||r_c||^2 of the latest evaluated iterate
    int64_t iter;        // index of the iterate the next cycle kernel reads
    int64_t done_cycle;  // first c that met the tolerance (or went non-finite); -1 otherwise
    int32_t status;      // 0 running, 1 converged, 2 non-finite
    uint32_t arrive;     // workgroups of the current kernel that have posted a partial
};

enum : int32_t { ST_RUNNING = 0, ST_CONVERGED = 1, ST_NONFINITE = 2 };

// ---------------------------------------------------------------------------
// Tile partition along one axis (subdomains of Sec. 3.3, overlap of Sec. 3.5).
// n points, tile t, overlap o (0 <= o < t).  n <= t: one tile of n points.
// Otherwise tiles start every t - o points; the last starts at n - t.
// ---------------------------------------------------------------------------
__host__ __device__ inline int axis_count(int n, int t, int o)
{
    return n <= t ? 1 : (n - o + (t - o) - 1) / (t - o);
}

__host__ __device__ inline int axis_origin(int n, int t, int o, int i)
{
    if (n <= t) return 0;
    const int st = i * (t - o);
    return st > n - t ? n - t : st;
}

// First point tile i writes back: the midpoint (rounded up) of its overlap
// with tile i - 1; the left neighbour keeps the lower half.
__host__ __device__ inline int axis_own_begin(int n, int t, int o, int i)
{
    if (i == 0) return 0;
    const int ext = n < t ? n : t;
    const int a = axis_origin(n, t, o, i);
    const int shared_pts = axis_origin(n, t, o, i - 1) + ext - a;
    return a + (shared_pts + 1) / 2;
}

__host__ __device__ inline int axis_own_end(int n, int t, int o, int i, int count)
{
    return i == count - 1 ? n : axis_own_begin(n, t, o, i + 1);
}

// ---------------------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Give every XCD a contiguous run of tiles so neighbouring tiles, which read
// each other's edge points as halo, share that XCD's L2.
// ---------------------------------------------------------------------------
__device__ inline int xcd_tile(int b, int nb)
{
    constexpr int kXcd = 8;
    const int q = nb / kXcd, r = nb % kXcd;
    const int k = b % kXcd, local = b / kXcd;
    const int base = k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q;
    return base + local;
}

// ---------------------------------------------------------------------------
// Deterministic sums: 64-lane butterfly, then waves in index order.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NT>
__device__ inline double block_sum(double v, double *red /* NT/64 doubles of LDS */)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();  // red may still be in use by a previous call
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    return t;  // identical in every thread
}

// Decide convergence for iterate c from its squared residual norm.
__device__ inline void judge(Ctrl *ctrl, int64_t c, double rsq, double tol)
{
    if (c == 0) ctrl->r0sq = rsq;
    const double r0sq = ctrl->r0sq;
    ctrl->last_rsq = rsq;
    const double rel = r0sq > 0.0 ? sqrt(rsq) / sqrt(r0sq) : 0.0;
    if (ctrl->status == ST_RUNNING) {
        if (!isfinite(rsq)) {
            ctrl->status = ST_NONFINITE;
            ctrl->done_cycle = c;
        } else if (rel <= tol) {
            ctrl->status = ST_CONVERGED;
            ctrl->done_cycle = c;
        }
    }
    ctrl->iter = c + 1;
}

// Every workgroup posts its partial sum of squares; the last one to arrive
// adds the partials in index order and judges iterate c (c < 0: ctrl->iter).
template <int NT>
__device__ inline void grid_finalize(double mine, double *partials, Ctrl *ctrl, int64_t c,
                                     double tol)
{
    __shared__ double red[NT / 64];
    __shared__ int last;
    const double bs = block_sum<NT>(mine, red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = bs;
        const unsigned prev = __hip_atomic_fetch_add(&ctrl->arrive, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double acc = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += NT) acc += partials[i];
    const double tot = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) {
        judge(ctrl, c < 0 ? ctrl->iter : c, tot, tol);
        ctrl->arrive = 0u;
    }
}

}  // namespace hj
