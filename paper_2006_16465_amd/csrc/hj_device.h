// hj_device.h -- device-side building blocks shared by the HIP kernels:
// the control block of a solve, the tile partition, the XCD-aware block
// mapping and the deterministic FP64 residual reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hj {

// Device-resident state of one solve.  Cycle kernels reduce the residual of
// the iterate they read and judge it on the device (see Red below), so the
// host only polls this block now and then.
struct Ctrl {
    double r0sq;         // ||r_0||^2
    double last_rsq;     // ||r_c||^2 of the latest judged iterate
    int64_t iter;        // one past the latest judged iterate
    int64_t done_cycle;  // first c that met the tolerance (or went non-finite); -1 otherwise
    int64_t stop_at;     // cycle kernels evaluating iterate k >= stop_at return at once
    int32_t status;      // 0 running, 1 converged, 2 non-finite, 3 stopped at max_cycles, 4 switch
    int32_t pad;
    // Optional hand-over point (sw_tol < 0: none).  The first iterate c with
    // a relative residual <= sw_tol (and above the tolerance) ends the solve
    // with ST_SWITCH if c >= sw_min_c; otherwise the solve runs on to the
    // tolerance.  The decision is taken once: sw_tol is set to -1 after it.
    double sw_tol;
    int64_t sw_min_c;
};

enum : int32_t { ST_RUNNING = 0, ST_CONVERGED = 1, ST_NONFINITE = 2, ST_LIMIT = 3, ST_SWITCH = 4 };

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

// Decide convergence for iterate c from its squared residual norm.  Once a
// verdict stands the block is frozen, so last_rsq stays that of done_cycle.
__device__ inline void judge(Ctrl *ctrl, int64_t c, double rsq, double tol)
{
    if (ctrl->status != ST_RUNNING) return;
    if (c == 0) ctrl->r0sq = rsq;
    const double r0sq = ctrl->r0sq;
    ctrl->last_rsq = rsq;
    ctrl->iter = c + 1;
    const double rel = r0sq > 0.0 ? sqrt(rsq) / sqrt(r0sq) : 0.0;
    int32_t st = ST_RUNNING;
    if (!isfinite(rsq)) st = ST_NONFINITE;
    else if (rel <= tol) st = ST_CONVERGED;
    else if (ctrl->sw_tol >= 0.0 && rel <= ctrl->sw_tol) {
        if (c >= ctrl->sw_min_c) st = ST_SWITCH;
        else ctrl->sw_tol = -1.0;
    }
    if (st != ST_RUNNING) {
        ctrl->done_cycle = c;
        // workgroups of the judging kernel (it evaluates iterate c + 1) that
        // start after the verdict return at once, as do all later kernels
        __hip_atomic_store(&ctrl->stop_at, c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Early exit of a cycle kernel that evaluates iterate k.  After a verdict on
// iterate c, iterate c + 1 is whole (the kernel that wrote it judged c - 1,
// which did not stop the solve); iterate c + 2 may be partial.
__device__ inline bool stopped(const Ctrl *ctrl, int64_t k)
{
    return k >= __hip_atomic_load(&ctrl->stop_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t read_status(const Ctrl *ctrl)
{
    return __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Residual bookkeeping handed to every kernel that reduces ||r||^2.
// Each workgroup stores its partial sum in part_cur[blockIdx.x] with a plain
// store.  The sum over the grid is formed by workgroup 0 of the NEXT kernel on
// the stream (the kernel boundary makes the partials visible), which judges
// iterate c - 1; no atomics and no cache-flushing fences inside the grid.
struct Red {
    double *part_cur;         // this kernel's partials (one per workgroup)
    const double *part_prev;  // the previous kernel's partials
    Ctrl *ctrl;
    int64_t c;                // index of the iterate this kernel evaluates
    int nb_prev;              // workgroups of the previous kernel (0: nothing to judge)
};

// Sum n partials in a fixed order and judge iterate c (one workgroup).
// Thread t adds chunks of 8 consecutive partials; 4 chunks (32 loads) are in
// flight per thread before any add, so a 64-lane workgroup reads 16K partials
// in a few memory latencies instead of one latency per partial.
template <int NT>
__device__ inline void judge_partials(const double *part, int n, Ctrl *ctrl, int64_t c, double tol)
{
    __shared__ double red[NT / 64];
    constexpr int V = 8, U = 4;
    double acc = 0.0;
    for (int base = 0; base < n; base += NT * V * U) {
        double v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i0 = base + (u * NT + (int)threadIdx.x) * V;
            if (i0 + V <= n) {
#pragma unroll
                for (int e = 0; e < V; ++e) v[u][e] = part[i0 + e];
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) v[u][e] = i0 + e < n ? part[i0 + e] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) acc += v[u][e];
    }
    const double tot = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) judge(ctrl, c, tot, tol);
}

template <int NT>
__device__ inline void post_partial(double mine, double *part_cur)
{
    __shared__ double red[NT / 64];
    const double bs = block_sum<NT>(mine, red);
    if (threadIdx.x == 0) part_cur[blockIdx.x] = bs;
}

}  // namespace hj
