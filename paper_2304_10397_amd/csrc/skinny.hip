// skinny.hip -- C -= A B for the updates inside the recursive panel
// factorization (Sec. III-A: the right half of a panel is updated with the
// factors of its left half): A is m x k with m the panel's full height (up to
// the matrix order) and k = 16, 32 or 64, B is k x n with n <= k, C is m x n.
//
// Such a product moves 16 m n + 8 m k bytes for 2 m n k flops: with k <= 64 it
// is bound by HBM, not by the matrix cores.  The general GEMM tiles it into
// 64- or 128-row tiles of 64 or more columns and stages every k-slab through
// LDS, a pipeline built for k = 512 that here runs one or two stages per tile
// with half of each tile's columns empty.  This kernel instead gives each wave
// 16-row blocks of C in turn: B, the same for every block, is laid out in LDS
// once per workgroup as MFMA fragments (lane-contiguous, so that the fragment
// reads are free of bank conflicts); per block the wave loads its A rows
// and C rows straight into registers (lanes 0-15 of a load take 16
// consecutive rows of one column: one 128-byte segment), runs the k/4
// v_mfma_f64_16x16x4_f64 steps per 16-column tile, and stores C.
//
// The product is computed transposed, C^T -= B^T A^T, so that each register
// of a lane's result is one element of a column and the loads and stores of C
// are column segments: MFMA lane l supplies B(4s + l/16, 16c + l%16) and
// A(r0 + l%16, 4s + l/16), and result register q of lane l is
// C(r0 + l%16, 16c + l/16 + 4q).
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kSkThreads = 256;
constexpr int kSkWaves = kSkThreads / 64;

template <int K>
__global__ __launch_bounds__(kSkThreads) void gemm_skinny_kernel(int64_t m, int n, const double *__restrict__ A,
                                                                   int64_t lda, const double *__restrict__ B,
                                                                   int64_t ldb, double *__restrict__ C, int64_t ldc)
{
    constexpr int NT = K / 16;  // 16-column tiles of C
    constexpr int S = K / 4;    // MFMA steps
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * kSkWaves + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * kSkWaves;

    // -B as MFMA fragments in LDS, bs[c][s][lane] (zero past column n; the
    // address is clamped so that every load is issued unconditionally)
    __shared__ double bs[NT][S][64];
    for (int e = threadIdx.x; e < NT * S * 64; e += kSkThreads) {
        const int l = e & 63, cs = e >> 6, c = cs / S, s = cs - c * S;
        const int col = 16 * c + (l & 15);
        const bool ok = col < n;
        const double x = B[off(4 * s + (l >> 4), ok ? col : n - 1, ldb)];
        bs[c][s][l] = ok ? -x : 0.0;
    }
    __syncthreads();

    const int64_t nblk = (m + 15) / 16;
    for (int64_t blk = wave; blk < nblk; blk += nwaves) {
        // the fragments are read from LDS in every block rather than hoisted
        // into registers (which would cost 2 k VGPRs per lane and occupancy)
        asm volatile("" ::: "memory");
        const int64_t r = blk * 16 + li;
        const bool rok = r < m;
        const int64_t rr = rok ? r : m - 1;
        double af[S];
#pragma unroll
        for (int s = 0; s < S; ++s) af[s] = A[off(rr, 4 * s + lg, lda)];
        dbl4 acc[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int col = 16 * c + lg + 4 * q;
                acc[c][q] = C[off(rr, col < n ? col : n - 1, ldc)];
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int c = 0; c < NT; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(bs[c][s][lane], af[s], acc[c], 0, 0, 0);
        }
        if (rok) {
#pragma unroll
            for (int c = 0; c < NT; ++c) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int col = 16 * c + lg + 4 * q;
                    if (col < n) C[off(r, col, ldc)] = acc[c][q];
                }
            }
        }
    }
}

template <int K>
int launch_k(int64_t m, int n, const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
             hipStream_t st)
{
    // enough waves to keep every CU's loads in flight, each then walking the
    // 16-row blocks grid-stride
    const int64_t nblk = (m + 15) / 16;
    int64_t g = (nblk + kSkWaves - 1) / kSkWaves;
    const int64_t cap = 256 * 4;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(gemm_skinny_kernel<K>, dim3((unsigned)g), dim3(kSkThreads), 0, st, m, n, A, lda, B, ldb, C,
                       ldc);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace

bool gemm_skinny_ok(int64_t n, int64_t k)
{
    return (k == 16 || k == 32 || k == 64) && n >= 1 && n <= k;
}

int launch_gemm_skinny(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double *C, int64_t ldc, hipStream_t st)
{
    if (m <= 0 || n <= 0) return HPL_OK;
    if (!gemm_skinny_ok(n, k)) return HPL_ERR_INTERNAL;
    switch (k) {
    case 16: return launch_k<16>(m, (int)n, A, lda, B, ldb, C, ldc, st);
    case 32: return launch_k<32>(m, (int)n, A, lda, B, ldb, C, ldc, st);
    default: return launch_k<64>(m, (int)n, A, lda, B, ldb, C, ldc, st);
    }
}

}  // namespace hplx
