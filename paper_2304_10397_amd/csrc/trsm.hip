// trsm.hip -- U12 <- L11^{-1} A12 (the DTRSM of the UPDATE phase, Sec. I /
// Sec. II: the pivoted rows of the block row are solved with the unit-lower
// triangle of the factored diagonal block).
//
// B is nbk x ncols (nbk <= 512), L is nbk x nbk unit lower.  One workgroup of
// 8 waves owns 64 columns of B for the whole solve; the 64 columns live in
// MFMA accumulators (32 row blocks of 16 rows x 4 column blocks of 16, row
// block rb owned by wave rb % 8).  Step i:
//   1. the owner of row block i hands its 16 x 64 block to LDS,
//   2. all 512 threads finish it by substitution with the 16 x 16 diagonal
//      block of L (so exactly representable data stay exact): each column's 16
//      rows sit in 16 lanes of one wave and x_k travels by lane shuffle; the
//      solved rows go to global memory,
//   3. every wave subtracts L[rb, i] * X_i from its row blocks rb > i with
//      v_mfma_f64_4x4x4_4b_f64 (the fast FP64 MFMA form on gfx950): the four
//      blocks b of one instruction take rows 16rb+4b..+3 of -L (lane l holds
//      -L[16rb + l%16][l/16], fetched from L2 one step ahead) and the same
//      4 columns of X_i (from LDS), so lane d accumulates
//      (row 16rb + 4((d>>2)&3) + (d>>4), column 4J + (d&3)) for column group J.
// Each column's arithmetic is independent of which workgroup holds it, so a
// split of the columns (look-ahead) gives identical bits.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kTrWB = 64;      // columns per workgroup
constexpr int kTrCG = kTrWB / 4;   // 4-column groups
constexpr int kTrWaves = 8;    // waves per workgroup
constexpr int kTrMaxRB = 32;   // row blocks (nbk <= 512)
constexpr int kTrQ = kTrMaxRB / kTrWaves;  // row blocks per wave

__global__ __launch_bounds__(kTrWaves * 64, 2) void trsm_llnu_kernel(const double *__restrict__ L, int64_t ldl,
                                                                    double *__restrict__ B, int64_t ldb, int nbk,
                                                                    int64_t ncols)
{
    __shared__ double Xs[2][16][kTrWB + 1];
    __shared__ double Ls[2][16][17];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * kTrWB;
    const int64_t crem = ncols - c0;
    const int nrb = (nbk + 15) >> 4;

    // lane d of accumulator (q, J): row 16rb + dr, column 4J + (d&3)
    const int dr = 4 * ((lane >> 2) & 3) + (lane >> 4);
    double acc[kTrQ][kTrCG];
#pragma unroll
    for (int q = 0; q < kTrQ; ++q) {
        const int rb = wave + kTrWaves * q;
        const int rr = 16 * rb + dr;
#pragma unroll
        for (int J = 0; J < kTrCG; ++J) {
            const int cc = 4 * J + (lane & 3);
            // unconditional load from clamped (always valid) indexes, then the mask
            const int rc = rr < nbk ? rr : nbk - 1;
            const int64_t ccc = cc < crem ? cc : crem - 1;
            const double v = B[off(rc, c0 + ccc, ldb)];
            acc[q][J] = (rb < nrb && rr < nbk && cc < crem) ? v : 0.0;
        }
    }

    // Next step's operands are fetched as soon as the current step's MFMAs are
    // issued, so their latency hides behind the next step's publish, barrier
    // and substitution: the diagonal block of L (one
    // element per thread of the upper half of the workgroup) and this wave's A
    // fragments (L[rb, i], 4 k-steps per row block, negated at use).
    double lsp = 0.0;
    double afr[kTrQ][4];
    auto fetch = [&](int i, double &ls, double (&af)[kTrQ][4]) {
        if (t >= 256) {
            const int e = t - 256, r = e & 15, c = e >> 4;
            const int gr = 16 * i + r, gc = 16 * i + c;
            const double v = L[off(gr < nbk ? gr : nbk - 1, gc < nbk ? gc : nbk - 1, ldl)];
            ls = (i < nrb && gr < nbk && gc < nbk) ? v : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kTrQ; ++q) {
            const int rb = wave + kTrWaves * q;
            const int lr = 16 * rb + (lane & 15);
#pragma unroll
            for (int k4 = 0; k4 < 4; ++k4) {
                const int kc = 4 * k4 + (lane >> 4);
                // raw L value, loaded unconditionally from clamped indexes
                // (in range wherever the fragment is used); the sign and the
                // row mask are applied at the MFMA
                const int lc = 16 * i + kc;
                af[q][k4] = L[off(lr < nbk ? lr : nbk - 1, lc < nbk ? lc : nbk - 1, ldl)];
            }
        }
    };
    fetch(0, lsp, afr);

    for (int i = 0; i < nrb; ++i) {
        const int par = i & 1;
        // 1. owner publishes row block i; the upper half stages the diagonal block of L
        if (wave == (i % kTrWaves)) {
            const int q = i / kTrWaves;
#pragma unroll
            for (int qq = 0; qq < kTrQ; ++qq) {
                if (qq != q) continue;
#pragma unroll
                for (int J = 0; J < kTrCG; ++J) Xs[par][dr][4 * J + (lane & 3)] = acc[qq][J];
            }
        }
        if (t >= 256) {
            const int e = t - 256;
            Ls[par][e & 15][e >> 4] = lsp;
        }
        __syncthreads();
        // 2. substitution of the 16 x kTrWB block: thread -> (row r, columns c, c + 32);
        //    a column's 16 rows sit in 16 consecutive lanes, so x_k is a lane shuffle
        {
            const int r = t & 15, c = t >> 4;
#pragma unroll
            for (int h = 0; h < kTrWB / 32; ++h) {
                const int cc = c + 32 * h;
                double x = Xs[par][r][cc];
#pragma unroll
                for (int kk = 0; kk < 15; ++kk) {
                    const double xk = __shfl(x, (lane & ~15) | kk, 64);
                    if (r > kk) x = __fma_rn(-Ls[par][r][kk], xk, x);
                }
                Xs[par][r][cc] = x;
                const int gr = 16 * i + r;
                if (gr < nbk && cc < crem) B[off(gr, c0 + cc, ldb)] = x;
            }
        }
        __syncthreads();
        // 3. trailing row blocks
#pragma unroll
        for (int q = 0; q < kTrQ; ++q) {
            const int rb = wave + kTrWaves * q;
            if (rb > i && rb < nrb) {
                const bool row_ok = 16 * rb + (lane & 15) < nbk;
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const int kc = 4 * k4 + (lane >> 4);
                    const double a = row_ok ? -afr[q][k4] : 0.0;  // -L[rb, i] fragment
#pragma unroll
                    for (int J = 0; J < kTrCG; ++J) {
                        const double b = Xs[par][kc][4 * J + (lane & 3)];
                        acc[q][J] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[q][J], 0, 0, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);  // bound the B fragments kept live
                }
            }
        }
        fetch(i + 1, lsp, afr);
    }
}

// Small TRSM (the panel's inner solves: nbk <= 64 RPL, few columns).  One wave
// per column of B: lane l holds rows l, l+64, l+128, ... of that column, and
// step k broadcasts the finished x_k with v_readlane (k is uniform), so the
// dependency chain per step is a readlane and an FMA.  The 4 waves of a
// workgroup share L, staged through LDS 16 columns at a time (double-buffered:
// the next chunk is fetched into registers while the current one is used).
// T = double (FP64 factorization, RPL = 4) or float (the mixed-precision
// factorization's FP32 panel, RPL = 8).
__device__ __forceinline__ double lane_value(double v, int l) { return read_lane(v, l); }
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
constexpr int kSmRPL = 4;    // rows per lane of the FP64 form (nbk <= 256)
constexpr int kSmRPL32 = 8;  // rows per lane of the FP32 form (nbk <= 512)
constexpr int kSmChunk = 16; // columns of L per LDS stage
// (FP32 only: with mx, the largest |x| of the solution is folded into *mx, the
// bit pattern of a non-negative float.)
template <typename T, int kSmRPL>
__global__ __launch_bounds__(256) void trsm_small_kernel(const T *__restrict__ L, int64_t ldl, T *__restrict__ B,
                                                         int64_t ldb, int nbk, int64_t ncols, unsigned *__restrict__ mx)
{
    __shared__ float red[4];
    __shared__ T Lc[2][kSmChunk][64 * kSmRPL + 1];  // Lc[buf][kk][r] = L(r, chunk*16 + kk)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t col = (int64_t)blockIdx.x * 4 + wave;
    const bool live = col < ncols;
    T x[kSmRPL];
#pragma unroll
    for (int s = 0; s < kSmRPL; ++s) {
        const int r = lane + 64 * s;
        x[s] = (live && r < nbk) ? B[off(r, col, ldb)] : (T)0;
    }
    const int nchunk = (nbk + kSmChunk - 1) / kSmChunk;
    // each thread fetches 4 RPL of the 16 x 64 RPL chunk entries: column kk = t / 16, rows (t % 16) + 16e
    constexpr int kPre = 4 * kSmRPL;
    T pre[kPre];
    auto fetch = [&](int ch) {
        const int kk = t >> 4, r0 = t & 15;
        const int gc = ch * kSmChunk + kk;
#pragma unroll
        for (int e = 0; e < kPre; ++e) {
            const int r = r0 + 16 * e;
            pre[e] = (gc < nbk && r < nbk) ? L[off(r, gc, ldl)] : (T)0;
        }
    };
    auto stash = [&](int buf) {
        const int kk = t >> 4, r0 = t & 15;
#pragma unroll
        for (int e = 0; e < kPre; ++e) Lc[buf][kk][r0 + 16 * e] = pre[e];
    };
    fetch(0);
    stash(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) fetch(ch + 1);
        const int kend = (nbk - ch * kSmChunk) < kSmChunk ? (nbk - ch * kSmChunk) : kSmChunk;
        // the step's L entries are read unconditionally and the update is a
        // select, so that the LDS reads of the next steps can be issued ahead
#pragma unroll 4
        for (int kk = 0; kk < kend; ++kk) {
            const int k = ch * kSmChunk + kk;
            const int sk = k >> 6, lk = k & 63;
            T xs = x[0];
#pragma unroll
            for (int s = 1; s < kSmRPL; ++s)
                if (sk == s) xs = x[s];
            const T xk = lane_value(xs, lk);
#pragma unroll
            for (int s = 0; s < kSmRPL; ++s) {
                const int r = lane + 64 * s;
                const T y = __fma_rn(-Lc[buf][kk][r], xk, x[s]);
                x[s] = r > k ? y : x[s];
            }
        }
        if (ch + 1 < nchunk) stash(buf ^ 1);
        __syncthreads();
    }
    if (live) {
#pragma unroll
        for (int s = 0; s < kSmRPL; ++s) {
            const int r = lane + 64 * s;
            if (r < nbk) B[off(r, col, ldb)] = x[s];
        }
    }
    if constexpr (sizeof(T) == 4) {
        if (mx) {  // uniform
            float am = 0.0f;
            if (live) {
#pragma unroll
                for (int s = 0; s < kSmRPL; ++s)
                    if (lane + 64 * s < nbk) am = fmaxf(am, fabsf((float)x[s]));
            }
            for (int o = 32; o > 0; o >>= 1) am = fmaxf(am, __shfl_xor(am, o, 64));
            if (lane == 0) red[wave] = am;
            __syncthreads();
            if (t == 0) atomicMax(mx, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
        }
    }
}

}  // namespace

int launch_trsm_llnu(const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nbk, int64_t ncols,
                     hipStream_t st)
{
    if (nbk <= 0 || ncols <= 0) return HPL_OK;
    if (nbk <= 64 * kSmRPL && ncols <= 4096) {
        const int64_t g = (ncols + 3) / 4;
        hipLaunchKernelGGL((trsm_small_kernel<double, kSmRPL>), dim3((unsigned)g), dim3(256), 0, st, L, ldl, B, ldb,
                           (int)nbk, ncols, nullptr);
        HPLX_TRY_LAUNCH();
        return HPL_OK;
    }
    if (nbk > 16 * kTrMaxRB) return HPL_ERR_INTERNAL;
    const int64_t g = (ncols + kTrWB - 1) / kTrWB;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(trsm_llnu_kernel, dim3((unsigned)g), dim3(kTrWaves * 64), 0, st, L, ldl, B, ldb, (int)nbk,
                       ncols);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

bool trsm32_small_ok(int64_t nbk, int64_t ncols)
{
    return nbk > 0 && nbk <= 64 * kSmRPL32 && ncols <= 4096;
}

int launch_trsm32_small(const float *L, int64_t ldl, float *B, int64_t ldb, int64_t nbk, int64_t ncols,
                        hipStream_t st, unsigned *mx)
{
    if (nbk <= 0 || ncols <= 0) return HPL_OK;
    if (!trsm32_small_ok(nbk, ncols)) return HPL_ERR_INTERNAL;
    const int64_t g = (ncols + 3) / 4;
    hipLaunchKernelGGL((trsm_small_kernel<float, kSmRPL32>), dim3((unsigned)g), dim3(256), 0, st, L, ldl, B, ldb,
                       (int)nbk, ncols, mx);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
