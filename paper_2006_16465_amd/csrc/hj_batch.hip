// hj_batch.hip -- many independent problems (2D and 1D, uneven sizes) solved
// together: one launch per cycle covers the work list of every problem.
//
// Per cycle c (cycle index kept in device memory, so a captured graph can
// replay a fixed sequence of launches):
//   k_batch_cycle2d  every 2D tile of every running problem (one launch for
//                    problems with hx == hy, one for the rest): one cycle of
//                    Sec. 4.1 from buffer c & 1 into the other, residual of
//                    the incoming iterate fused into the load (per-tile
//                    partial sums);
//   k_batch_cycle1d  the same for the 1D tile groups (Sec. 3.3);
//   k_batch_judge    per problem, the partial sums of iterate c in a fixed
//                    order, and the verdict;
//   k_batch_advance  c += 1.
// The verdict on iterate c lands before cycle c + 1 starts, so a converged
// problem's iterate c (buffer c & 1) is never overwritten: two buffers per
// problem suffice (the caller's x and one scratch array).  The tile bodies are
// the ones the single-problem kernels run (hj_tiles.h), so every problem's
// iterates equal those of its own single-problem solve bit for bit.
//
// One workgroup per work item, handed out XCD by XCD in list order (problems
// in turn, tiles row-major), rather than a grid-stride loop over the list:
// the loop kept about 30 more VGPRs live around the tile body (154 against
// 124 at 64x64 FP64), one wave per SIMD fewer.  Items of problems that have
// stopped return after reading the problem's status.
#include <hip/hip_runtime.h>

#include "hj_launch.h"
#include "hj_tiles.h"

namespace hj {
namespace {

template <int NT>
__device__ __forceinline__ void post_partial_at(double mine, double *slot)
{
    __shared__ double red[NT / 64];
    const double bs = block_sum<NT>(mine, red);
    if (threadIdx.x == 0) *slot = bs;
}

template <typename T, int C, int R, int W, bool ISO>
__global__ __launch_bounds__(64 * W) void k_batch_cycle2d(const BProb *__restrict__ probs,
                                                          const int32_t *__restrict__ owner,
                                                          int64_t nitems, const BCtl *bc,
                                                          const Ctrl *ctrl, double *part,
                                                          int64_t npart, int s)
{
    constexpr int NT = 64 * W;
    const int64_t c = bc->cycle;
    double *pc = part + (c & 1) * npart;
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const int p = owner[w];
    if (read_status(&ctrl[p]) != ST_RUNNING) return;
    const BProb &P = probs[p];
    const T *f = (const T *)P.f;
    const T *xin = (const T *)((c & 1) ? P.s1 : P.x);
    T *xout = (T *)((c & 1) ? P.x : P.s1);
    const int tile = (int)(w - P.item0);
    const double rsq = reg_tile_2d<T, C, R, W, true, ISO, rotate_rows<T>()>(P.g2, tile, f, xin, xout, s);
    post_partial_at<NT>(rsq, &pc[P.part0 + tile]);
}

template <typename T, int TT>
__global__ __launch_bounds__(kNT) void k_batch_cycle1d(const BProb *__restrict__ probs,
                                                       const int32_t *__restrict__ owner,
                                                       int64_t nitems, const BCtl *bc,
                                                       const Ctrl *ctrl, double *part,
                                                       int64_t npart, int s)
{
    const int64_t c = bc->cycle;
    double *pc = part + (c & 1) * npart;
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const int p = owner[w];
    if (read_status(&ctrl[p]) != ST_RUNNING) return;
    const BProb &P = probs[p];
    const T *f = (const T *)P.f;
    const T *xin = (const T *)((c & 1) ? P.s1 : P.x);
    T *xout = (T *)((c & 1) ? P.x : P.s1);
    const int64_t blk = w - P.item0;
    const double rsq = lds_tiles_1d<T, TT, true>(P.g1, blk, f, xin, xout, s);
    post_partial_at<kNT>(rsq, &pc[P.part0 + blk]);
}

// One wavefront per problem: partials of iterate c summed lane-strided in
// index order, then a fixed butterfly; lane 0 judges against the problem's
// own tolerance.  With tol <= 0 it never converges and stops at its own
// max_cycles.
__global__ __launch_bounds__(256) void k_batch_judge(const BProb *__restrict__ probs, int nprob,
                                                     const BCtl *bc, Ctrl *ctrl,
                                                     const double *part, int64_t npart)
{
    const int lane = (int)threadIdx.x & 63;
    const int p = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    if (p >= nprob) return;
    if (read_status(&ctrl[p]) != ST_RUNNING) return;
    const int64_t c = bc->cycle;
    const double *base = part + (c & 1) * npart + probs[p].part0;
    const int64_t n = probs[p].nitems;
    double acc = 0.0;
    for (int64_t i = lane; i < n; i += 64) acc += base[i];
    acc = wave_sum(acc);
    if (lane == 0) {
        Ctrl *k = &ctrl[p];
        judge(k, c, acc, probs[p].tol);
        if (k->status == ST_RUNNING && c >= probs[p].max_cycles) {
            k->done_cycle = c;
            __hip_atomic_store(&k->status, (int32_t)ST_LIMIT, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_batch_advance(BCtl *bc)
{
    if (threadIdx.x == 0) bc->cycle = bc->cycle + 1;
}

__global__ __launch_bounds__(256) void k_batch_init(Ctrl *ctrl, int nprob, BCtl *bc,
                                                    int64_t max_cycles)
{
    for (int p = (int)(blockIdx.x * blockDim.x + threadIdx.x); p < nprob;
         p += (int)(gridDim.x * blockDim.x)) {
        Ctrl k{};
        k.done_cycle = -1;
        k.stop_at = INT64_MAX;
        k.status = ST_RUNNING;
        ctrl[p] = k;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bc->cycle = 0;
        bc->max_cycles = max_cycles;
    }
}

// Problems whose final iterate sits in the scratch buffer (odd index) copy it
// into the caller's x.  Grid: (problem, chunk).
template <typename T>
__global__ __launch_bounds__(256) void k_batch_finalize(const BProb *__restrict__ probs,
                                                        const Ctrl *ctrl)
{
    const int p = (int)blockIdx.x;
    const int64_t fin = ctrl[p].done_cycle;
    if (fin < 0 || (fin & 1) == 0) return;
    const BProb &P = probs[p];
    const int64_t nx = P.dim == 2 ? P.g2.nx : P.g1.n;
    const int64_t ny = P.dim == 2 ? P.g2.ny : 1;
    const int64_t ld = P.dim == 2 ? P.g2.ld : P.g1.n;
    const T *src = (const T *)P.s1;
    T *dst = (T *)P.x;
    const int64_t total = nx * ny;
    for (int64_t i = (int64_t)blockIdx.y * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.y * 256) {
        const int64_t r = i / nx, q = i - r * nx;
        dst[r * ld + q] = src[r * ld + q];
    }
}

template <typename T, int TX, int TY, bool ISO>
hipError_t bcyc2(const BatchLaunch &L, hipStream_t st)
{
    using S = RegShape<TX, TY>;
    k_batch_cycle2d<T, S::C, S::R, S::W, ISO><<<(unsigned)L.nitems, 64 * S::W, 0, st>>>(
        L.probs, L.owner, L.nitems, L.bc, L.ctrl, L.part, L.npart, L.s);
    return hipGetLastError();
}

template <typename T, int TT>
hipError_t bcyc1(const BatchLaunch &L, hipStream_t st)
{
    k_batch_cycle1d<T, TT><<<(unsigned)L.nitems, kNT, 0, st>>>(L.probs, L.owner, L.nitems, L.bc, L.ctrl,
                                                               L.part, L.npart, L.s);
    return hipGetLastError();
}

#define HJ_BATCH_TILES2(X) X(32, 16) X(32, 32) X(32, 64) X(32, 128) X(64, 16) X(64, 32) X(64, 64) X(64, 128)

template <typename T>
hipError_t bcyc2_t(int tx, int ty, bool iso, const BatchLaunch &L, hipStream_t st)
{
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return iso ? bcyc2<T, a, b, true>(L, st) : bcyc2<T, a, b, false>(L, st);
    HJ_BATCH_TILES2(HJ_TILE)
#undef HJ_TILE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t bcyc1_t(int t, const BatchLaunch &L, hipStream_t st)
{
    switch (t) {
    case 32: return bcyc1<T, 32>(L, st);
    case 64: return bcyc1<T, 64>(L, st);
    case 128: return bcyc1<T, 128>(L, st);
    case 256: return bcyc1<T, 256>(L, st);
    case 512: return bcyc1<T, 512>(L, st);
    case 1024: return bcyc1<T, 1024>(L, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- refinement
constexpr int kRBX = 64, kRRPT = 8;  // 2D blocks: 64 columns x (4 x 8) rows
constexpr int kR1 = 2048;           // 1D block: 256 threads x 8 points

// r = f - A x in FP64 (the oracle's residual association), stored as FP32;
// the correction starts from zero; this thread's share of ||r||^2.
__device__ double ref_resid_block(const BRef &P, int64_t blk)
{
    double rsq = 0.0;
    if (P.dim == 2) {
        const int gx = (P.nx + kRBX - 1) / kRBX;
        const int by = (int)(blk / gx), bx = (int)(blk - (int64_t)by * gx);
        const int c = bx * kRBX + (int)(threadIdx.x % kRBX);
        const int rbeg = (by * 4 + (int)(threadIdx.x / kRBX)) * kRRPT;
        if (c < P.nx && rbeg < P.ny) {
            const int64_t ld = P.ld;
            const double *x = P.x;
            double up = rbeg > 0 ? x[(int64_t)(rbeg - 1) * ld + c] : 0.0;
            double cen = x[(int64_t)rbeg * ld + c];
            for (int i = 0; i < kRRPT; ++i) {
                const int r = rbeg + i;
                if (r >= P.ny) break;
                const int64_t a = (int64_t)r * ld + c;
                const double dn = r + 1 < P.ny ? x[a + ld] : 0.0;
                const double w = c > 0 ? x[a - 1] : 0.0;
                const double e = c + 1 < P.nx ? x[a + 1] : 0.0;
                const double rr = res2(P.f[a], cen, w, e, up, dn, P.wx, P.wy);
                const int64_t a32 = (int64_t)r * P.nx + c;
                P.r32[a32] = (float)rr;
                P.e32[a32] = 0.0f;
                rsq += rr * rr;
                up = cen;
                cen = dn;
            }
        }
    } else {
        const int64_t n = P.nx;
        const int64_t i0 = blk * kR1 + threadIdx.x;
        for (int j = 0; j < kR1 / kNT; ++j) {
            const int64_t i = i0 + (int64_t)j * kNT;
            if (i >= n) break;
            const double w = i > 0 ? P.x[i - 1] : 0.0;
            const double e = i + 1 < n ? P.x[i + 1] : 0.0;
            const double rr = res1(P.f[i], P.x[i], w, e, P.wx);
            P.r32[i] = (float)rr;
            P.e32[i] = 0.0f;
            rsq += rr * rr;
        }
    }
    return rsq;
}

__global__ __launch_bounds__(kNT) void k_batch_ref_resid(const BRef *__restrict__ refs,
                                                         const int32_t *__restrict__ owner,
                                                         int64_t nitems, double *part)
{
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const BRef &P = refs[owner[w]];
    const int64_t blk = w - P.item0;
    const double rsq = ref_resid_block(P, blk);
    post_partial_at<kNT>(rsq, &part[P.part0 + blk]);
}

__global__ __launch_bounds__(256) void k_batch_ref_norm(const BRef *__restrict__ refs, int nref,
                                                        const double *part, double *rsq)
{
    const int lane = (int)threadIdx.x & 63;
    const int p = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
    if (p >= nref) return;
    const double *base = part + refs[p].part0;
    const int64_t n = refs[p].nitems;
    double acc = 0.0;
    for (int64_t i = lane; i < n; i += 64) acc += base[i];
    acc = wave_sum(acc);
    if (lane == 0) rsq[p] = acc;
}

__global__ __launch_bounds__(kNT) void k_batch_ref_axpy(const BRef *__restrict__ refs,
                                                        const int32_t *__restrict__ owner,
                                                        int64_t nitems)
{
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nitems) return;
    const BRef &P = refs[owner[w]];
    const int64_t blk = w - P.item0;
    if (P.dim == 2) {
        const int gx = (P.nx + kRBX - 1) / kRBX;
        const int by = (int)(blk / gx), bx = (int)(blk - (int64_t)by * gx);
        const int c = bx * kRBX + (int)(threadIdx.x % kRBX);
        const int rbeg = (by * 4 + (int)(threadIdx.x / kRBX)) * kRRPT;
        if (c >= P.nx) return;
        for (int i = 0; i < kRRPT; ++i) {
            const int r = rbeg + i;
            if (r >= P.ny) break;
            double *xp = &P.x[(int64_t)r * P.ld + c];
            *xp = *xp + (double)P.e32[(int64_t)r * P.nx + c];
        }
    } else {
        const int64_t i0 = blk * kR1 + threadIdx.x;
        for (int j = 0; j < kR1 / kNT; ++j) {
            const int64_t i = i0 + (int64_t)j * kNT;
            if (i >= P.nx) break;
            P.x[i] = P.x[i] + (double)P.e32[i];
        }
    }
}

}  // namespace

int64_t ref_items(int dim, int64_t nx, int64_t ny)
{
    if (dim == 2) return ((nx + kRBX - 1) / kRBX) * ((ny + 4 * kRRPT - 1) / (4 * kRRPT));
    return (nx + kR1 - 1) / kR1;
}

hipError_t launch_batch_ref_resid(const BRef *refs, const int32_t *owner, int64_t nitems, double *part,
                                  hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    k_batch_ref_resid<<<(unsigned)nitems, kNT, 0, st>>>(refs, owner, nitems, part);
    return hipGetLastError();
}

hipError_t launch_batch_ref_norm(const BRef *refs, int nref, const double *part, double *rsq,
                                 hipStream_t st)
{
    k_batch_ref_norm<<<(unsigned)((nref + 3) / 4), 256, 0, st>>>(refs, nref, part, rsq);
    return hipGetLastError();
}

hipError_t launch_batch_ref_axpy(const BRef *refs, const int32_t *owner, int64_t nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    k_batch_ref_axpy<<<(unsigned)nitems, kNT, 0, st>>>(refs, owner, nitems);
    return hipGetLastError();
}

bool batch2d_supported(int tx, int ty)
{
#define HJ_TILE(a, b) \
    if (tx == a && ty == b) return true;
    HJ_BATCH_TILES2(HJ_TILE)
#undef HJ_TILE
    return false;
}

hipError_t launch_batch_cycle2d(int dt, int tx, int ty, bool iso, const BatchLaunch &L, hipStream_t st)
{
    if (L.nitems <= 0) return hipSuccess;
    return dt == F64 ? bcyc2_t<double>(tx, ty, iso, L, st) : bcyc2_t<float>(tx, ty, iso, L, st);
}

hipError_t launch_batch_cycle1d(int dt, int t, const BatchLaunch &L, hipStream_t st)
{
    if (L.nitems <= 0) return hipSuccess;
    return dt == F64 ? bcyc1_t<double>(t, L, st) : bcyc1_t<float>(t, L, st);
}

hipError_t launch_batch_judge(const BProb *probs, int nprob, const BCtl *bc, Ctrl *ctrl,
                              const double *part, int64_t npart, hipStream_t st)
{
    k_batch_judge<<<(unsigned)((nprob + 3) / 4), 256, 0, st>>>(probs, nprob, bc, ctrl, part, npart);
    return hipGetLastError();
}

hipError_t launch_batch_advance(BCtl *bc, hipStream_t st)
{
    k_batch_advance<<<1, 64, 0, st>>>(bc);
    return hipGetLastError();
}

hipError_t launch_batch_init(Ctrl *ctrl, int nprob, BCtl *bc, int64_t max_cycles, hipStream_t st)
{
    const unsigned nb = (unsigned)((nprob + 255) / 256);
    k_batch_init<<<nb > 0 ? nb : 1, 256, 0, st>>>(ctrl, nprob, bc, max_cycles);
    return hipGetLastError();
}

hipError_t launch_batch_finalize(int dt, const BProb *probs, int nprob, const Ctrl *ctrl,
                                 hipStream_t st)
{
    const dim3 grid((unsigned)nprob, 16);
    if (dt == F64) k_batch_finalize<double><<<grid, 256, 0, st>>>(probs, ctrl);
    else k_batch_finalize<float><<<grid, 256, 0, st>>>(probs, ctrl);
    return hipGetLastError();
}

}  // namespace hj
