// grad.hip -- the matrix gradient of a linear solve.
//
// For X = A^{-1} B and a loss with gradient W = dL/dX, the adjoint of the
// solve is grad_B = A^{-T} W (a transposed solve with the saved factors) and
// grad_A = -grad_B X^T, a rank-nrhs outer product that fills all n^2 entries.
// With nrhs small (16 in the differentiable-solve workload) that product is
// bound by writing grad_A (8 n^2 bytes) and by FP64 FMA issue (2 n^2 nrhs
// flops), so it is one pass that writes every entry exactly once:
//   * a workgroup of 256 threads owns 256 rows x kGaCols columns; thread t
//     keeps its row of grad_B (kGaK values at a time) in registers;
//   * the kGaCols rows of X it needs are staged in LDS (a broadcast read per
//     wave);
//   * each wave stores 64 consecutive rows of one column per instruction.
// Sums run over the right-hand sides in ascending order (FMA), then negate.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kGaThreads = 256;
constexpr int kGaCols = 32;  // columns of grad_A per workgroup
constexpr int kGaK = 16;     // right-hand sides held in registers at a time

__global__ __launch_bounds__(kGaThreads) void grad_a_kernel(const double *__restrict__ G, int64_t ldg,
                                                            const double *__restrict__ X, int64_t ldx, int64_t n,
                                                            int64_t k, double *__restrict__ D, int64_t ldd)
{
    __shared__ double xs[kGaK][kGaCols];  // xs[r][c] = X(j0 + c, r0 + r)
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kGaThreads + t;
    const int64_t j0 = (int64_t)blockIdx.y * kGaCols;
    const int ncols = (int)((n - j0) < kGaCols ? (n - j0) : kGaCols);
    const bool live = i < n;
    double acc[kGaCols];
#pragma unroll
    for (int c = 0; c < kGaCols; ++c) acc[c] = 0.0;
    for (int64_t r0 = 0; r0 < k; r0 += kGaK) {
        const int nr = (int)((k - r0) < kGaK ? (k - r0) : kGaK);
        __syncthreads();
        for (int e = t; e < kGaK * kGaCols; e += kGaThreads) {
            const int c = e % kGaCols, r = e / kGaCols;
            xs[r][c] = (c < ncols && r < nr) ? X[off(j0 + c, r0 + r, ldx)] : 0.0;
        }
        double g[kGaK];
#pragma unroll
        for (int r = 0; r < kGaK; ++r) g[r] = (live && r < nr) ? G[off(i, r0 + r, ldg)] : 0.0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kGaCols; ++c)
#pragma unroll
            for (int r = 0; r < kGaK; ++r) acc[c] = __fma_rn(g[r], xs[r][c], acc[c]);
    }
    if (!live) return;
#pragma unroll
    for (int c = 0; c < kGaCols; ++c)
        if (c < ncols) D[off(i, j0 + c, ldd)] = 0.0 - acc[c];  // +0 when nrhs = 0
}

}  // namespace

int launch_grad_a(const double *G, int64_t ldg, const double *X, int64_t ldx, int64_t n, int64_t k, double *D,
                  int64_t ldd, hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    const int64_t gx = (n + kGaThreads - 1) / kGaThreads, gy = (n + kGaCols - 1) / kGaCols;
    if (gx > 0x7fffffffll || gy > 65535) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(grad_a_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kGaThreads), 0, st, G, ldg, X, ldx, n,
                       k, D, ldd);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
