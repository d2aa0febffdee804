// solve.hip -- triangular solves with the factors (Sec. II: after A = P L U,
// A x = b becomes U x = L^{-1} P^{-1} b and x follows by applying U^{-1}).
//
// The solve reads the n x n factors once (HBM-bound, 2 n^2 nrhs flops), but its
// rows depend on each other, so it is organized as a sweep over diagonal blocks
// of kBs = 64 rows with ONE launch per block:
//   * every workgroup of the launch first finishes the diagonal block itself:
//     each wave takes up to 4 right-hand sides at a time (their recurrences
//     interleaved), lane r holds x_r, and x_k reaches the other lanes by
//     shuffle -- no barrier, no second launch.  Every workgroup reads the
//     block's rows of B, so the finished rows are stored only by the last
//     workgroup to have read them (a counter that returns to zero at the end
//     of each launch), never while another workgroup may still read them;
//   * then the workgroup subtracts the block's contribution from its share of
//     the rows not yet solved, one row per thread (a skinny GEMV: for L and U
//     the row's values are read coalesced across lanes; for the transposed
//     operators each lane reads a contiguous column segment).  All 64 values
//     of a row are loaded at once and reused for every right-hand side.
// mode 0: L unit lower, forward.  mode 1: U upper, backward.
// mode 2: U^T (lower, diagonal u_ii), forward.  mode 3: L^T unit upper, backward.
//
// Interchanges on B: all chunk plans (see laswp.hip) are computed by one
// launch in parallel, then one workgroup applies them in order (or in reverse
// order for A^T X = B).
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kBs = 64;          // diagonal block rows (one per lane)
constexpr int kSvThreads = 256;  // 4 waves
constexpr int kSvChain = 4;      // right-hand sides per wave in the diagonal block

template <int mode, typename TT>
__global__ __launch_bounds__(kSvThreads) void solve_block_kernel(const TT *__restrict__ T, int64_t ldt,
                                                                 double *__restrict__ B, int64_t ldb, int64_t nrhs,
                                                                 int64_t r0, int bs, int64_t row_begin,
                                                                 int64_t row_end, unsigned *__restrict__ done)
{
    __shared__ double Td[kBs][kBs + 1];  // Td[r][c] = T(r0 + r, r0 + c), identity-padded past bs
    __shared__ int last;
    extern __shared__ double Y[];        // [nrhs][kBs] solved block
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    constexpr bool lower = (mode == 0 || mode == 2);
    constexpr bool unit = (mode == 0 || mode == 3);
    constexpr bool tr = (mode >= 2);

    // ---- 1. diagonal block: stage it (coalesced; all loads issued before the
    //      first LDS store, so the staging costs one memory round trip), then
    //      one wave per right-hand side
    constexpr int kStage = kBs * kBs / kSvThreads;
    static_assert(kBs * kBs % kSvThreads == 0, "staging must divide evenly");
    double sv[kStage];
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
        const int e = t + q * kSvThreads, r = e % kBs, c = e / kBs;
        const bool in = r < bs && c < bs;
        const double v = (double)load_or(in, T + off(r0 + r, r0 + c, ldt), T + off(r0, r0, ldt), (TT)0);
        sv[q] = in ? v : (r == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
        const int e = t + q * kSvThreads;
        Td[e % kBs][e / kBs] = sv[q];
    }
    __syncthreads();
    // each wave carries kSvChain consecutive right-hand sides through the same
    // step loop (independent recurrences, interleaved)
    for (int64_t c0 = (int64_t)wid * kSvChain; c0 < nrhs; c0 += (int64_t)kSvChain * (kSvThreads / 64)) {
        double x[kSvChain];
#pragma unroll
        for (int j = 0; j < kSvChain; ++j) {
            const bool ok = lane < bs && c0 + j < nrhs;
            x[j] = load_or(ok, B + off(r0 + lane, c0 + j, ldb), B + off(r0, c0, ldb), 0.0);
        }
        const int64_t left = nrhs - c0;
        // one step of the recurrence of chain value xj, k the step's row
        auto step = [&](double &xj, int k, bool below, double a, double dkk) __attribute__((always_inline)) {
            double xk = read_lane(xj, k);
            if (!unit) xk = xk / dkk;
            if (lane == k) xj = xk;
            if (below) xj = __fma_rn(-a, xk, xj);
        };
        if (left >= kSvChain) {  // all chains live (uniform in the wave): interleaved
#pragma unroll 4
            for (int s = 0; s < kBs; ++s) {
                const int k = lower ? s : kBs - 1 - s;
                const bool below = lower ? (lane > k) : (lane < k);
                const double a = tr ? Td[k][lane] : Td[lane][k];  // T_op(lane, k)
                const double dkk = Td[k][k];
#pragma unroll
                for (int j = 0; j < kSvChain; ++j) step(x[j], k, below, a, dkk);
            }
        } else {  // the last few right-hand sides: one chain at a time
#pragma unroll
            for (int j = 0; j < kSvChain; ++j) {
                if (j >= left) break;
                double xj = x[j];
#pragma unroll 8
                for (int s = 0; s < kBs; ++s) {
                    const int k = lower ? s : kBs - 1 - s;
                    const bool below = lower ? (lane > k) : (lane < k);
                    const double a = tr ? Td[k][lane] : Td[lane][k];
                    step(xj, k, below, a, Td[k][k]);
                }
                x[j] = xj;
            }
        }
#pragma unroll
        for (int j = 0; j < kSvChain; ++j)
            if (lane < bs && c0 + j < nrhs) Y[(c0 + j) * kBs + lane] = x[j];
    }
    // every load of the block's rows of B has been consumed above; the last
    // workgroup to arrive stores the solved rows (the counter wraps to zero)
    __syncthreads();
    if (t == 0) {
        if (gridDim.x == 1) {
            last = 1;
        } else {
            __threadfence();
            last = atomicInc(done, gridDim.x - 1) == gridDim.x - 1;
        }
    }
    __syncthreads();
    if (last) {
        for (int64_t e = t; e < nrhs * kBs; e += kSvThreads) {
            const int r = (int)(e % kBs);
            if (r < bs) B[off(r0 + r, e / kBs, ldb)] = Y[e];
        }
    }
    if (row_end <= row_begin) return;

    // ---- 2. update of this workgroup's rows: one row per thread; the row's kBs
    //      operator values are loaded in one burst (independent loads, one
    //      round trip) and reused for every right-hand side, whose solved
    //      block values are LDS broadcasts
    const int64_t i = row_begin + (int64_t)blockIdx.x * kSvThreads + t;
    if (i >= row_end) return;
    double a[kBs];
    if (mode < 2) {
        const TT *base = T + off(i, r0, ldt);  // T_op(i, r0 + k) = T(i, r0 + k)
#pragma unroll
        for (int k = 0; k < kBs; ++k) a[k] = (double)load_or(k < bs, base + (size_t)k * (size_t)ldt, base, (TT)0);
    } else {
        const TT *base = T + off(r0, i, ldt);  // T_op(i, r0 + k) = T(r0 + k, i)
#pragma unroll
        for (int k = 0; k < kBs; ++k) a[k] = (double)load_or(k < bs, base + k, base, (TT)0);
    }
    for (int64_t c = 0; c < nrhs; ++c) {
        const double *y = Y + c * kBs;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kBs; ++k) acc += a[k] * y[k];
        B[off(i, c, ldb)] -= acc;
    }
}

// Applies the chunk plans in order (reverse = 0) or reverse order to B's columns.
constexpr int kApThreads = 1024;
constexpr int kApRhs = 16;
__global__ __launch_bounds__(kApThreads) void apply_plans_seq_kernel(double *__restrict__ B, int64_t ldb,
                                                                     int64_t nrhs, const int32_t *__restrict__ plans,
                                                                     int64_t nchunks, int reverse)
{
    __shared__ double vals[2 * kMaxSwaps * kApRhs];
    const int t = threadIdx.x;
    for (int64_t qq = 0; qq < nchunks; ++qq) {
        const int64_t q = reverse ? nchunks - 1 - qq : qq;
        const int32_t *rows = plans + (size_t)q * kPlanStride;
        const int32_t *src = rows + 2 * kMaxSwaps;
        const int ns = rows[4 * kMaxSwaps];
        for (int64_t c0 = 0; c0 < nrhs; c0 += kApRhs) {
            const int nr = (int)((nrhs - c0) < kApRhs ? (nrhs - c0) : kApRhs);
            for (int e = t; e < ns * nr; e += kApThreads) {
                const int s = e % ns, c = e / ns;
                vals[c * 2 * kMaxSwaps + s] = B[off(rows[s], c0 + c, ldb)];
            }
            __syncthreads();
            for (int e = t; e < ns * nr; e += kApThreads) {
                const int s = e % ns, c = e / ns;
                const int ss = src[s];
                if (ss != s) B[off(rows[s], c0 + c, ldb)] = vals[c * 2 * kMaxSwaps + ss];
            }
            __syncthreads();
        }
    }
}

}  // namespace

int launch_solve_block(const double *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs, int64_t r0, int64_t bs,
                       int64_t row_begin, int64_t row_end, int mode, unsigned *done, hipStream_t st)
{
    if (bs <= 0 || nrhs <= 0) return HPL_OK;
    if (bs > kBs) return HPL_ERR_INTERNAL;
    const int64_t rows = row_end > row_begin ? row_end - row_begin : 0;
    const int64_t per = (int64_t)kSvThreads;  // one row per thread
    int64_t g = (rows + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    const size_t lds = sizeof(double) * (size_t)kBs * (size_t)nrhs;
    if (lds > 64 * 1024) return HPL_ERR_INTERNAL;
    switch (mode) {
    case 0:
        hipLaunchKernelGGL((solve_block_kernel<0, double>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb, nrhs,
                           r0, (int)bs, row_begin, row_end, done);
        break;
    case 1:
        hipLaunchKernelGGL((solve_block_kernel<1, double>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb, nrhs,
                           r0, (int)bs, row_begin, row_end, done);
        break;
    case 2:
        hipLaunchKernelGGL((solve_block_kernel<2, double>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb, nrhs,
                           r0, (int)bs, row_begin, row_end, done);
        break;
    case 3:
        hipLaunchKernelGGL((solve_block_kernel<3, double>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb, nrhs,
                           r0, (int)bs, row_begin, row_end, done);
        break;
    default: return HPL_ERR_INTERNAL;
    }
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

// FP32 factors (the mixed-precision LU), FP64 right-hand sides: modes 0 and 1.
int launch_solve_block_f32(const float *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs, int64_t r0, int64_t bs,
                           int64_t row_begin, int64_t row_end, int mode, unsigned *done, hipStream_t st)
{
    if (bs <= 0 || nrhs <= 0) return HPL_OK;
    if (bs > kBs) return HPL_ERR_INTERNAL;
    const int64_t rows = row_end > row_begin ? row_end - row_begin : 0;
    int64_t g = (rows + kSvThreads - 1) / kSvThreads;
    if (g < 1) g = 1;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    const size_t lds = sizeof(double) * (size_t)kBs * (size_t)nrhs;
    if (lds > 64 * 1024) return HPL_ERR_INTERNAL;
    if (mode == 0)
        hipLaunchKernelGGL((solve_block_kernel<0, float>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb,
                           nrhs, r0, (int)bs, row_begin, row_end, done);
    else if (mode == 1)
        hipLaunchKernelGGL((solve_block_kernel<1, float>), dim3((unsigned)g), dim3(kSvThreads), lds, st, T, ldt, B, ldb,
                           nrhs, r0, (int)bs, row_begin, row_end, done);
    else
        return HPL_ERR_INTERNAL;
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_apply_plans_seq(double *B, int64_t ldb, int64_t nrhs, const int32_t *plans, int64_t nchunks, bool reverse,
                           hipStream_t st)
{
    if (nchunks <= 0 || nrhs <= 0) return HPL_OK;
    hipLaunchKernelGGL(apply_plans_seq_kernel, dim3(1), dim3(kApThreads), 0, st, B, ldb, nrhs, plans, nchunks,
                       reverse ? 1 : 0);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

// The whole solve on stream st: interchanges on B (A X = B: first; A^T X = B:
// last, in reverse order), then per chunk of at most 64 right-hand sides the
// forward and the backward sweep of 64-row diagonal blocks.
int solve_sequence(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n, int64_t lda,
                   int64_t ldb, int trans, int32_t *plans, int *pivot_err, unsigned *done, hipStream_t st)
{
    const int64_t bs = kBs;
    const int64_t rhs_chunk = 64;
    const int64_t nchunks = (n + kMaxSwaps - 1) / kMaxSwaps;
    auto swaps = [&](bool reverse) -> int {
        HPLX_PROPAGATE(launch_swap_plans_all(ipiv, n, 0, n, reverse, plans, pivot_err, st));
        return launch_apply_plans_seq(B, ldb, nrhs, plans, nchunks, reverse, st);
    };
    auto sweep = [&](int mode, double *Bc, int64_t nr) -> int {
        const bool fwd = (mode == 0 || mode == 2);
        const int64_t nblk = (n + bs - 1) / bs;
        for (int64_t q = 0; q < nblk; ++q) {
            const int64_t r0 = (fwd ? q : nblk - 1 - q) * bs;
            const int64_t b = (n - r0) < bs ? (n - r0) : bs;
            const int64_t rb = fwd ? r0 + b : 0, re = fwd ? n : r0;
            HPLX_PROPAGATE(launch_solve_block(LU, lda, Bc, ldb, nr, r0, b, rb, re, mode, done, st));
        }
        return HPL_OK;
    };
    if (trans == 0) HPLX_PROPAGATE(swaps(false));
    for (int64_t c0 = 0; c0 < nrhs; c0 += rhs_chunk) {
        const int64_t nr = (nrhs - c0) < rhs_chunk ? (nrhs - c0) : rhs_chunk;
        double *Bc = B + off(0, c0, ldb);
        if (trans == 0) {
            HPLX_PROPAGATE(sweep(0, Bc, nr));
            HPLX_PROPAGATE(sweep(1, Bc, nr));
        } else {
            HPLX_PROPAGATE(sweep(2, Bc, nr));
            HPLX_PROPAGATE(sweep(3, Bc, nr));
        }
    }
    if (trans == 1) HPLX_PROPAGATE(swaps(true));
    return HPL_OK;
}

// U X = B alone (the back substitution of an augmented system, whose
// right-hand sides already hold L^{-1} P^{-1} B): per chunk of at most 64
// right-hand sides, the backward sweep of 64-row diagonal blocks.
int solve_upper_sequence(const double *U, double *B, int64_t nrhs, int64_t n, int64_t lda, int64_t ldb, unsigned *done,
                         hipStream_t st)
{
    const int64_t bs = kBs;
    const int64_t rhs_chunk = 64;
    const int64_t nblk = (n + bs - 1) / bs;
    for (int64_t c0 = 0; c0 < nrhs; c0 += rhs_chunk) {
        const int64_t nr = (nrhs - c0) < rhs_chunk ? (nrhs - c0) : rhs_chunk;
        double *Bc = B + off(0, c0, ldb);
        for (int64_t q = nblk - 1; q >= 0; --q) {
            const int64_t r0 = q * bs;
            const int64_t b = (n - r0) < bs ? (n - r0) : bs;
            HPLX_PROPAGATE(launch_solve_block(U, lda, Bc, ldb, nr, r0, b, 0, r0, 1, done, st));
        }
    }
    return HPL_OK;
}

}  // namespace hplx
