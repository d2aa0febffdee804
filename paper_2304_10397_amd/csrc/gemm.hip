// gemm.hip -- FP64 MFMA rank-k update C(m x n) -= A(m x k) * B(k x n).
//
// This is the UPDATE-phase DGEMM (the rank-NB update of the trailing matrix,
// Sec. I / Sec. II), where nearly all of the flops of the method are spent.
// At NB = 512 its arithmetic intensity is NB/8 = 64 flop per byte of C
// traffic, far above the MI355X ridge (78.6 TFLOP/s / 8 TB/s ~ 9.8), so the
// kernel is bound by the FP64 matrix cores.
//
// gfx950 design
//  * FP64 MFMA: v_mfma_f64_4x4x4_4b_f64.  On gfx950 the four-block 4x4x4 form
//    sustains ~72 TFLOP/s in a pure issue loop, against ~47 for the
//    16x16x4 form (both measured on the hardware), so the kernel is built on
//    it.  The instruction holds 4 independent blocks b: lane 16k+4b+i supplies
//    A_b(i,k), lane 16k+4b+j supplies B_b(k,j), and lane 16i+4b+j holds
//    D_b(i,j) (layout checked on the hardware).  All four blocks get the same
//    4-row slice of A (the A value depends only on lane%4 and lane/16) and
//    consecutive 4-column slices of B, so one instruction updates a 4 x 16
//    strip: lane d holds C(4I + d/16, 16G + d%16) for row group I, column
//    group G.
//  * Block tile BM x BN, K staged BK = 16 at a time through double-buffered
//    LDS (one barrier per stage); each wave owns a (BM/WM) x (BN/WN) sub-tile
//    of accumulators that stay in registers for the whole K loop.
//  * Accumulators live in AGPRs (so the A/B operands do not compete with them
//    for VGPR read ports) and start from zero; the epilogue applies
//    C <- C - acc a column group at a time.  Every element is therefore
//    C - sum_k a_ik b_kj with the same k order and the same instruction
//    whatever the tiling -- the look-ahead split of the update reproduces the
//    unsplit update bit for bit.
//  * Workgroups are dispatched round-robin over the 8 XCDs (each with its own
//    L2).  The block index is remapped so that each XCD receives a contiguous
//    run of tiles, and tiles are ordered in groups of kGroupM tile-rows so the
//    workgroups resident on one XCD share A row-panels and B column-panels in
//    that XCD's L2.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int BK = 16;
constexpr int kGroupM = 8;

template <int BM, int BN, int WM, int WN>
struct GemmCfg {
    static constexpr int NT = WM * WN * 64;
    static constexpr int TM = BM / WM;   // rows per wave
    static constexpr int TN = BN / WN;   // cols per wave
    static constexpr int FI = TM / 4;    // 4-row groups per wave
    static constexpr int FG = TN / 16;   // 16-column groups per wave
    static constexpr int APAD = 4;
    static constexpr int BPAD = 4;
    static constexpr int AL = BM * BK / NT;  // A doubles loaded per thread per stage
    static constexpr int BL = BK * BN / NT;  // B doubles loaded per thread per stage
    static_assert(TM % 4 == 0 && TN % 16 == 0, "wave tile: rows multiple of 4, columns of 16");
    static_assert((BM * BK) % NT == 0 && (BK * BN) % NT == 0, "loads must divide evenly");
};

// Block index -> (tile_m, tile_n): XCD-contiguous runs, then grouped ordering.
__device__ __forceinline__ void tile_of_block(int64_t bid, int64_t nwg, int64_t tiles_m, int64_t tiles_n,
                                              int64_t &tm, int64_t &tn)
{
    const int64_t xcd = bid & 7, in_xcd = bid >> 3;
    const int64_t per = nwg >> 3, rem = nwg & 7;
    const int64_t lin = xcd * per + (xcd < rem ? xcd : rem) + in_xcd;
    const int64_t group_size = (int64_t)kGroupM * tiles_n;
    const int64_t g = lin / group_size;
    const int64_t first_m = g * kGroupM;
    const int64_t gm = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
    const int64_t r = lin - g * group_size;
    tm = first_m + r % gm;
    tn = r / gm;
}

template <int BM, int BN, int WM, int WN, int TRAIL>
__global__ __launch_bounds__(WM *WN * 64, 2) void gemm_sub_kernel(
    int64_t m, int64_t n, int64_t k, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t tiles_m,
    int64_t tiles_n)
{
    using Cfg = GemmCfg<BM, BN, WM, WN>;
    constexpr int NT = Cfg::NT, TM = Cfg::TM, TN = Cfg::TN, FI = Cfg::FI, FG = Cfg::FG;
    // Marks the kernel as using AGPRs, so the compiler selects the MFMA form with
    // accumulators in AGPRs: the A/B operands then have the VGPR read ports to
    // themselves instead of competing with the accumulator in the same banks.
    asm volatile("" ::: "a0");
    constexpr int AS = BM + Cfg::APAD, BS = BN + Cfg::BPAD;
    __shared__ double As[2][BK][AS];
    __shared__ double Bs[2][BK][BS];

    int64_t tm, tn;
    tile_of_block(blockIdx.x, (int64_t)gridDim.x, tiles_m, tiles_n, tm, tn);
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t mrem = m - m0, nrem = n - n0;

    // Per-thread global load coordinates (fixed over the K loop).
    // A: idx = t + NT*q -> row idx % BM = t % BM, kk = t / BM + (NT/BM)*q (rows contiguous across lanes).
    // B: idx = t + NT*q -> kk idx % BK = t % BK, col t / BK + (NT/BK)*q (k contiguous within a column).
    constexpr int AQ = NT / BM;  // k rows of A covered per q
    constexpr int BQ = NT / BK;  // columns of B covered per q
    const int a_r = t % BM, a_k = t / BM;
    const int b_k = t % BK, b_c = t / BK;
    const double *pa = A + off(m0 + a_r, a_k, lda);
    const double *pb = B + off(b_k, n0 + b_c, ldb);
    const int64_t a_step = (int64_t)AQ * lda, b_step = (int64_t)BQ * ldb;
    const bool a_row_ok = a_r < mrem;
    const bool full_mn = (mrem >= BM) && (nrem >= BN);
    double ra[Cfg::AL], rb[Cfg::BL];

    auto load_stage = [&](int64_t k0) {
        const int64_t krem = k - k0;
        const double *p = pa + (size_t)k0 * (size_t)lda;
        const double *q2 = pb + k0;
        if (full_mn && krem >= BK) {
#pragma unroll
            for (int q = 0; q < Cfg::AL; ++q) { ra[q] = *p; p += a_step; }
#pragma unroll
            for (int q = 0; q < Cfg::BL; ++q) { rb[q] = *q2; q2 += b_step; }
        } else {
#pragma unroll
            for (int q = 0; q < Cfg::AL; ++q) {
                ra[q] = (a_row_ok && a_k + AQ * q < krem) ? *p : 0.0;
                p += a_step;
            }
#pragma unroll
            for (int q = 0; q < Cfg::BL; ++q) {
                rb[q] = (b_c + BQ * q < nrem && b_k < krem) ? *q2 : 0.0;
                q2 += b_step;
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < Cfg::AL; ++q) As[buf][a_k + AQ * q][a_r] = ra[q];
#pragma unroll
        for (int q = 0; q < Cfg::BL; ++q) Bs[buf][b_k][b_c + BQ * q] = rb[q];
    };

    load_stage(0);

    // lane d accumulates element (wm*TM + 4I + d/16, wn*TN + 16G + d%16) of the tile
    double acc[FI][FG];
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int g = 0; g < FG; ++g) acc[i][g] = 0.0;
    const int crow0 = wm * TM + (lane >> 4);
    const int ccol0 = wn * TN + (lane & 15);

    store_stage(0);
    __syncthreads();

    const int nst = (int)((k + BK - 1) / BK);
    const int arow = wm * TM + (lane & 3);   // A value depends on lane%4 (row) and lane/16 (k)
    const int bcol = wn * TN + (lane & 15);
    const int kq = lane >> 4;
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) load_stage((int64_t)(s + 1) * BK);
#pragma unroll
        for (int k4 = 0; k4 < BK / 4; ++k4) {
            double bf[FG];
#pragma unroll
            for (int g = 0; g < FG; ++g) bf[g] = Bs[buf][4 * k4 + kq][bcol + 16 * g];
#pragma unroll
            for (int i = 0; i < FI; ++i) {
                const double af = As[buf][4 * k4 + kq][arow + 4 * i];
#pragma unroll
                for (int g = 0; g < FG; ++g)
                    acc[i][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(af, bf[g], acc[i][g], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);  // bound the fragments kept live across k-steps
        }
        if (s + 1 < nst) store_stage(buf ^ 1);
        __syncthreads();
    }

    // C <- C - acc, one 16-column group at a time (bounded live registers)
    double *pc = C + off(m0 + crow0, n0 + ccol0, ldc);
    const int64_t c_step = 16 * ldc;
#pragma unroll
    for (int g = 0; g < FG; ++g) {
        const bool col_ok = ccol0 + 16 * g < nrem;
        double *pcol = pc + (size_t)g * (size_t)c_step;
#pragma unroll
        for (int i = 0; i < FI; ++i)
            if (col_ok && crow0 + 4 * i < mrem) pcol[4 * i] = pcol[4 * i] - acc[i][g];
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int BM, int BN, int WM, int WN, int TRAIL>
int launch_cfg(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
               int64_t ldb, double *C, int64_t ldc, hipStream_t st)
{
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    const int64_t nwg = tiles_m * tiles_n;
    if (nwg > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL((gemm_sub_kernel<BM, BN, WM, WN, TRAIL>), dim3((unsigned)nwg), dim3(WM * WN * 64), 0, st,
                       m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace

// variant: 0 = auto, 1 = 128x128, 2 = 128x64, 3 = 64x64, 4 = 128x32; add kTrailing
// (launch_gemm_sub's caller passes variant | kTrailingFlag) for the trailing update.
int launch_gemm_sub(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                    int64_t ldb, double *C, int64_t ldc, int variant, hipStream_t st)
{
    if (m <= 0 || n <= 0 || k <= 0) return HPL_OK;
    const bool trail = (variant & kGemmTrailing) != 0;
    variant &= ~kGemmTrailing;
    if (variant == 0) {
        if (n <= 32)
            variant = 4;
        else if (n <= 64)
            variant = 2;
        else if (m * n < (int64_t)256 * 128 * 128)
            variant = 3;
        else
            variant = 1;
    }
    if (trail) {
        switch (variant) {
        case 1: return launch_cfg<128, 128, 2, 2, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        case 2: return launch_cfg<128, 64, 2, 2, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        case 3: return launch_cfg<64, 64, 2, 2, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        case 4: return launch_cfg<128, 32, 4, 1, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        default: return HPL_ERR_INTERNAL;
        }
    }
    switch (variant) {
    case 1: return launch_cfg<128, 128, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 2: return launch_cfg<128, 64, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 3: return launch_cfg<64, 64, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 4: return launch_cfg<128, 32, 4, 1, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    default: return HPL_ERR_INTERNAL;
    }
}

}  // namespace hplx
