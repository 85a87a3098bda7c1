// hj_refine.hip -- kernels of the mixed-precision solve: FP64 residual written
// in FP32 (which also clears the FP32 correction), FP64 correction
// accumulation.  The FP32 hierarchical
// cycles in between are the ordinary cycle kernels (hj_kernels.hip).
//
// Iterative refinement: r = f - A x in FP64; A e = r solved approximately by
// FP32 cycles from e = 0; x += e in FP64; repeat.  Because the cycle is a
// consistent stationary iteration (x' = x + K (f - A x)), restarting it on the
// correction equation continues the same iteration, so the cycle count to a
// tolerance matches the pure-FP64 solve while each cycle moves half the bytes.
#include <hip/hip_runtime.h>

#include "hj_launch.h"

namespace hj {
namespace {

constexpr int kBX = 64, kBY = 4, kRPT = 8;  // same column walk as the sweep kernel

// r32 = (float)(f - A x) with x, f in FP64; partial sums of ||f - A x||^2 (FP64);
// e32 = 0, the start of the next correction solve.
__global__ __launch_bounds__(256) void k_resid2d_f64_to_f32(Geom2 g, const double *__restrict__ f,
                                                            const double *__restrict__ x,
                                                            float *__restrict__ r32,
                                                            float *__restrict__ e32,
                                                            double *__restrict__ part)
{
    const int gx = (g.nx + kBX - 1) / kBX;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int by = b / gx, bx = b - by * gx;
    const int c = bx * kBX + (int)(threadIdx.x % kBX);
    const int rbeg = (by * kBY + (int)(threadIdx.x / kBX)) * kRPT;
    const int64_t ld = g.ld;
    double rsq = 0.0;
    if (c < g.nx && rbeg < g.ny) {
        double up = rbeg > 0 ? x[(int64_t)(rbeg - 1) * ld + c] : 0.0;
        double cen = x[(int64_t)rbeg * ld + c];
#pragma unroll
        for (int i = 0; i < kRPT; ++i) {
            const int r = rbeg + i;
            if (r < g.ny) {
                const int64_t a = (int64_t)r * ld + c;
                const double dn = r + 1 < g.ny ? x[a + ld] : 0.0;
                const double w = c > 0 ? x[a - 1] : 0.0;
                const double e = c + 1 < g.nx ? x[a + 1] : 0.0;
                const double rr = f[a] - (g.wx * ((2.0 * cen - w) - e) + g.wy * ((2.0 * cen - up) - dn));
                r32[a] = (float)rr;
                e32[a] = 0.0f;
                rsq += rr * rr;
                up = cen;
                cen = dn;
            }
        }
    }
    post_partial<256>(rsq, part);
}

// x += (double)e over the interior (pitched rows)
__global__ __launch_bounds__(256) void k_axpy_f32_to_f64(int nx, int ny, int64_t ld,
                                                         const float *__restrict__ e,
                                                         double *__restrict__ x)
{
    const int64_t total = (int64_t)nx * ny;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * 256) {
        const int64_t r = i / nx, c = i - r * nx;
        const int64_t a = r * ld + c;
        x[a] = x[a] + (double)e[a];
    }
}

unsigned stride_blocks(int nx, int ny)
{
    const int64_t total = (int64_t)nx * ny;
    const int64_t nb = (total + 255) / 256;
    return (unsigned)(nb < 8192 ? nb : 8192);
}

}  // namespace

int64_t resid2d_mixed_blocks(const Geom2 &g)
{
    const int64_t gx = (g.nx + kBX - 1) / kBX;
    const int64_t gy = (g.ny + kBY * kRPT - 1) / (kBY * kRPT);
    return gx * gy;
}

hipError_t launch_resid2d_f64_to_f32(const Geom2 &g, const double *f, const double *x, float *r32,
                                     float *e32, double *part, hipStream_t st)
{
    k_resid2d_f64_to_f32<<<(unsigned)resid2d_mixed_blocks(g), 256, 0, st>>>(g, f, x, r32, e32, part);
    return hipGetLastError();
}

hipError_t launch_axpy_f32_to_f64(const Geom2 &g, const float *e, double *x, hipStream_t st)
{
    k_axpy_f32_to_f64<<<stride_blocks(g.nx, g.ny), 256, 0, st>>>(g.nx, g.ny, g.ld, e, x);
    return hipGetLastError();
}


}  // namespace hj
