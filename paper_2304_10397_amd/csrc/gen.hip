// gen.hip -- random system generator and the HPL residual check.
//
// Generator: every element is an independent function of its linear index, so
// the residual can regenerate A tile by tile instead of keeping a copy of it
// (at N = 163840 the original A would need a second 215 GB).  The kernel is
// HBM-write bound: consecutive lanes write consecutive rows of one column.
//
// Residual: one thread per row; the thread walks the row j = 0..n-1 in order,
// accumulating sum_j a_ij x_j and sum_j |a_ij| (a_ij read, coalesced across
// the wave, or regenerated), then the wave/LDS reduction takes maxima and one
// atomicMax per workgroup publishes them (maxima of non-negative doubles
// commute with their uint64 bit patterns, so the result is order independent).
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kGenThreads = 256;
constexpr int kGenRowsPerThread = 4;

__global__ __launch_bounds__(kGenThreads) void generate_kernel(uint64_t s0, double *__restrict__ M,
                                                               int64_t rows, int64_t cols, int64_t ld)
{
    const int64_t rows_per_block = (int64_t)kGenThreads * kGenRowsPerThread;
    const int64_t r_base = (int64_t)blockIdx.x * rows_per_block + threadIdx.x;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        double *col = M + (size_t)j * (size_t)ld;
        const uint64_t cbase = (uint64_t)j * (uint64_t)rows;
#pragma unroll
        for (int q = 0; q < kGenRowsPerThread; ++q) {
            int64_t i = r_base + (int64_t)q * kGenThreads;
            if (i < rows) col[i] = gen_value(s0, cbase + (uint64_t)i);
        }
    }
}

// Standard normal values (the weights of the differentiable solve's loss):
// Box-Muller of the stream's outputs 2 idx and 2 idx + 1,
// z = sqrt(-2 ln(1 - u1)) cos(2 pi u2), u = (h >> 11) 2^-53 in [0, 1).
__device__ __forceinline__ double normal_value(uint64_t s0, uint64_t idx)
{
    const double u1 = (double)(sm64_mix(s0 + (2ull * idx + 1ull) * kGamma) >> 11) * 0x1.0p-53;
    const double u2 = (double)(sm64_mix(s0 + (2ull * idx + 2ull) * kGamma) >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925286766559 * u2);
}

__global__ __launch_bounds__(kGenThreads) void generate_normal_kernel(uint64_t s0, double *__restrict__ M,
                                                                      int64_t rows, int64_t cols, int64_t ld)
{
    const int64_t rows_per_block = (int64_t)kGenThreads * kGenRowsPerThread;
    const int64_t r_base = (int64_t)blockIdx.x * rows_per_block + threadIdx.x;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y) {
        double *col = M + (size_t)j * (size_t)ld;
        const uint64_t cbase = (uint64_t)j * (uint64_t)rows;
#pragma unroll
        for (int q = 0; q < kGenRowsPerThread; ++q) {
            int64_t i = r_base + (int64_t)q * kGenThreads;
            if (i < rows) col[i] = normal_value(s0, cbase + (uint64_t)i);
        }
    }
}

__global__ void add_diagonal_kernel(double *__restrict__ M, int64_t n, int64_t ld, double alpha)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) M[off(i, i, ld)] += alpha;
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t count, unsigned long long v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

constexpr int kResThreads = 256;
constexpr int kResRhs = 8;      // right-hand sides per pass
constexpr int kResChunk = 256;  // columns of x staged in LDS at a time

__device__ __forceinline__ unsigned long long dbits(double v)
{
    return (unsigned long long)__double_as_longlong(v);
}

// max that lets NaN win (NaN compares false, so keep it once seen)
__device__ __forceinline__ double nanmax(double a, double b)
{
    return (a != a || b != b) ? __longlong_as_double(0x7ff8000000000000ll) : (a > b ? a : b);
}

__device__ __forceinline__ double block_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = nanmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = sh[0];
    for (int w = 1; w < kResThreads / 64; ++w) r = nanmax(r, sh[w]);
    return r;
}

template <bool GEN>
__global__ __launch_bounds__(kResThreads) void residual_kernel(
    const double *__restrict__ A, int64_t lda, uint64_t s0, int64_t n,
    const double *__restrict__ X, int64_t ldx, const double *__restrict__ B, int64_t ldb,
    int64_t rhs0, int nr, bool do_anorm, unsigned long long *__restrict__ red)
{
    __shared__ double xs[kResChunk][kResRhs];
    __shared__ double sh[kResThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * kResThreads + threadIdx.x;
    const bool live = i < n;
    double dot[kResRhs];
#pragma unroll
    for (int c = 0; c < kResRhs; ++c) dot[c] = 0.0;
    double rsum = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kResChunk) {
        const int64_t jn = (n - j0) < kResChunk ? (n - j0) : kResChunk;
        __syncthreads();
        for (int t = threadIdx.x; t < kResChunk * kResRhs; t += kResThreads) {
            int jj = t % kResChunk, c = t / kResChunk;
            xs[jj][c] = (jj < jn && c < nr) ? X[off(j0 + jj, rhs0 + c, ldx)] : 0.0;
        }
        __syncthreads();
        if (live) {
            for (int jj = 0; jj < jn; ++jj) {
                const int64_t j = j0 + jj;
                double a = GEN ? gen_value(s0, (uint64_t)i + (uint64_t)j * (uint64_t)n)
                               : A[off(i, j, lda)];
                rsum += fabs(a);
#pragma unroll
                for (int c = 0; c < kResRhs; ++c) dot[c] += a * xs[jj][c];
            }
        }
    }
    if (do_anorm) {
        double m = block_max(live ? rsum : 0.0, sh);
        if (threadIdx.x == 0) atomicMax(&red[0], dbits(m));
    }
    for (int c = 0; c < nr; ++c) {
        double r = 0.0, xa = 0.0, ba = 0.0;
        if (live) {
            double b = B[off(i, rhs0 + c, ldb)];
            r = fabs(dot[c] - b);
            xa = fabs(X[off(i, rhs0 + c, ldx)]);
            ba = fabs(b);
        }
        double mr = block_max(r, sh);
        double mx = block_max(xa, sh);
        double mb = block_max(ba, sh);
        if (threadIdx.x == 0) {
            unsigned long long *slot = red + 1 + 3 * (rhs0 + c);
            atomicMax(&slot[0], dbits(mr));
            atomicMax(&slot[1], dbits(mx));
            atomicMax(&slot[2], dbits(mb));
        }
    }
}

}  // namespace

int launch_generate(uint64_t s0, double *M, int64_t rows, int64_t cols, int64_t ld, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return HPL_OK;
    const int64_t rows_per_block = (int64_t)kGenThreads * kGenRowsPerThread;
    int64_t gx = (rows + rows_per_block - 1) / rows_per_block;
    int64_t gy = cols < 65535 ? cols : 65535;
    if (gx > 0x7fffffff) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(generate_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kGenThreads), 0, st, s0,
                       M, rows, cols, ld);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_generate_normal(uint64_t s0, double *M, int64_t rows, int64_t cols, int64_t ld, hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return HPL_OK;
    const int64_t rows_per_block = (int64_t)kGenThreads * kGenRowsPerThread;
    int64_t gx = (rows + rows_per_block - 1) / rows_per_block;
    int64_t gy = cols < 65535 ? cols : 65535;
    if (gx > 0x7fffffff) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(generate_normal_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(kGenThreads), 0, st, s0,
                       M, rows, cols, ld);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_add_diagonal(double *M, int64_t n, int64_t ld, double alpha, hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    const int64_t g = (n + 255) / 256;
    if (g > 0x7fffffff) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(add_diagonal_kernel, dim3((unsigned)g), dim3(256), 0, st, M, n, ld, alpha);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v, hipStream_t st)
{
    if (count <= 0) return HPL_OK;
    int64_t g = (count + 255) / 256;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)g), dim3(256), 0, st, p, count, v);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_residual(const double *A, int64_t lda, bool gen, uint64_t s0, int64_t n, const double *X,
                    int64_t ldx, const double *B, int64_t ldb, int64_t nrhs, unsigned long long *red,
                    hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    const int64_t g = (n + kResThreads - 1) / kResThreads;
    for (int64_t r0 = 0; r0 < nrhs; r0 += kResRhs) {
        int nr = (int)((nrhs - r0) < kResRhs ? (nrhs - r0) : kResRhs);
        bool do_anorm = (r0 == 0);
        if (gen)
            hipLaunchKernelGGL(residual_kernel<true>, dim3((unsigned)g), dim3(kResThreads), 0, st, A, lda,
                               s0, n, X, ldx, B, ldb, r0, nr, do_anorm, red);
        else
            hipLaunchKernelGGL(residual_kernel<false>, dim3((unsigned)g), dim3(kResThreads), 0, st, A,
                               lda, s0, n, X, ldx, B, ldb, r0, nr, do_anorm, red);
        HPLX_TRY_LAUNCH();
    }
    return HPL_OK;
}

}  // namespace hplx
