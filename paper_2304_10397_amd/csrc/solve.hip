// solve.hip -- triangular solves with the factors (Sec. II: after A = P L U,
// A x = b becomes U x = L^{-1} P^{-1} b and x follows by applying U^{-1}).
//
// Blocked column sweep over diagonal blocks of bs rows:
//   trsv_block_kernel  one workgroup solves the bs x bs diagonal block for all
//                      right-hand sides (LDS-resident, one barrier per row);
//   gemv_update_kernel subtracts the block's contribution from the rows not
//                      yet solved.  Reading the factors once is the whole
//                      cost, so the kernel is HBM-bound: for L and U the
//                      column segments are read coalesced one row per lane;
//                      for the transposed solves a wave reads one column
//                      segment and reduces it with shuffles.
// mode 0: L unit lower, forward.  mode 1: U upper, backward.
// mode 2: U^T (lower, diagonal u_ii), forward.  mode 3: L^T unit upper, backward.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kSvBS = 64;      // diagonal block rows (max)
constexpr int kSvRhs = 16;     // right-hand sides per pass
constexpr int kSvThreads = 256;

// element (r, c) of the operator T_op of the mode, inside the diagonal block
__device__ __forceinline__ double top_elem(const double *T, int64_t ldt, int64_t r0, int r, int c, int mode)
{
    // modes 0,1 use T(r, c); modes 2,3 use T(c, r)
    return (mode < 2) ? T[off(r0 + r, r0 + c, ldt)] : T[off(r0 + c, r0 + r, ldt)];
}

__global__ __launch_bounds__(kSvThreads) void trsv_block_kernel(const double *__restrict__ T, int64_t ldt,
                                                                double *__restrict__ B, int64_t ldb, int64_t nrhs,
                                                                int64_t r0, int bs, int mode)
{
    __shared__ double Ts[kSvBS][kSvBS + 1];
    __shared__ double X[kSvBS][kSvRhs];
    __shared__ double Xo[kSvBS][kSvRhs];
    const int t = threadIdx.x;
    for (int e = t; e < bs * bs; e += kSvThreads) {
        const int r = e % bs, c = e / bs;
        Ts[r][c] = top_elem(T, ldt, r0, r, c, mode);
    }
    const bool lower = (mode == 0 || mode == 2);
    const bool unit = (mode == 0 || mode == 3);
    for (int64_t cr0 = 0; cr0 < nrhs; cr0 += kSvRhs) {
        const int nr = (int)((nrhs - cr0) < kSvRhs ? (nrhs - cr0) : kSvRhs);
        __syncthreads();
        for (int e = t; e < bs * kSvRhs; e += kSvThreads) {
            const int r = e % bs, c = e / bs;
            X[r][c] = (c < nr) ? B[off(r0 + r, cr0 + c, ldb)] : 0.0;
        }
        __syncthreads();
        for (int s = 0; s < bs; ++s) {
            const int kcol = lower ? s : bs - 1 - s;  // row being finished
            for (int e = t; e < bs * kSvRhs; e += kSvThreads) {
                const int r = e % bs, c = e / bs;
                double xk = X[kcol][c];
                if (!unit) xk = xk / Ts[kcol][kcol];
                if (r == kcol) Xo[r][c] = xk;
                const bool below = lower ? (r > kcol) : (r < kcol);
                if (below) X[r][c] = X[r][c] - Ts[r][kcol] * xk;
            }
            __syncthreads();
        }
        for (int e = t; e < bs * kSvRhs; e += kSvThreads) {
            const int r = e % bs, c = e / bs;
            if (c < nr) B[off(r0 + r, cr0 + c, ldb)] = Xo[r][c];
        }
    }
}

// rows [row_begin, row_end) of B -= T_op(rows, block) * X(block) where block = [r0, r0+bs).
__global__ __launch_bounds__(kSvThreads) void gemv_update_kernel(const double *__restrict__ T, int64_t ldt,
                                                                 double *__restrict__ B, int64_t ldb,
                                                                 int64_t nrhs, int64_t r0, int bs,
                                                                 int64_t row_begin, int64_t row_end, int mode)
{
    __shared__ double X[kSvBS][kSvRhs];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    for (int64_t cr0 = 0; cr0 < nrhs; cr0 += kSvRhs) {
        const int nr = (int)((nrhs - cr0) < kSvRhs ? (nrhs - cr0) : kSvRhs);
        __syncthreads();
        for (int e = t; e < bs * kSvRhs; e += kSvThreads) {
            const int r = e % bs, c = e / bs;
            X[r][c] = (c < nr) ? B[off(r0 + r, cr0 + c, ldb)] : 0.0;
        }
        __syncthreads();
        if (mode < 2) {
            // one row per thread; T(i, r0 + q) read coalesced across lanes
            const int64_t i = row_begin + (int64_t)blockIdx.x * kSvThreads + t;
            if (i < row_end) {
                double acc[kSvRhs];
#pragma unroll
                for (int c = 0; c < kSvRhs; ++c) acc[c] = 0.0;
                for (int q = 0; q < bs; ++q) {
                    const double a = T[off(i, r0 + q, ldt)];
#pragma unroll
                    for (int c = 0; c < kSvRhs; ++c) acc[c] += a * X[q][c];
                }
                for (int c = 0; c < nr; ++c) B[off(i, cr0 + c, ldb)] -= acc[c];
            }
        } else {
            // one row per wave; T(r0 + q, i) is a contiguous column segment
            const int64_t i = row_begin + (int64_t)blockIdx.x * (kSvThreads / 64) + wid;
            if (i < row_end) {
                double acc[kSvRhs];
#pragma unroll
                for (int c = 0; c < kSvRhs; ++c) acc[c] = 0.0;
                for (int q = lane; q < bs; q += 64) {
                    const double a = T[off(r0 + q, i, ldt)];
#pragma unroll
                    for (int c = 0; c < kSvRhs; ++c) acc[c] += a * X[q][c];
                }
#pragma unroll
                for (int c = 0; c < kSvRhs; ++c)
                    for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
                if (lane == 0)
                    for (int c = 0; c < nr; ++c) B[off(i, cr0 + c, ldb)] -= acc[c];
            }
        }
    }
}

}  // namespace

int launch_trsv_block(const double *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs, int64_t r0, int64_t bs,
                      int mode, hipStream_t st)
{
    if (bs <= 0 || nrhs <= 0) return HPL_OK;
    if (bs > kSvBS) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(trsv_block_kernel, dim3(1), dim3(kSvThreads), 0, st, T, ldt, B, ldb, nrhs, r0, (int)bs, mode);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_gemv_update(const double *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs, int64_t r0, int64_t bs,
                       int64_t row_begin, int64_t row_end, int mode, hipStream_t st)
{
    if (bs <= 0 || nrhs <= 0 || row_end <= row_begin) return HPL_OK;
    if (bs > kSvBS) return HPL_ERR_INTERNAL;
    const int64_t rows = row_end - row_begin;
    const int64_t per = (mode < 2) ? kSvThreads : kSvThreads / 64;
    const int64_t g = (rows + per - 1) / per;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(gemv_update_kernel, dim3((unsigned)g), dim3(kSvThreads), 0, st, T, ldt, B, ldb, nrhs, r0,
                       (int)bs, row_begin, row_end, mode);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
