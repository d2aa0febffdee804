// gemm.hip -- FP64 MFMA rank-k update C(m x n) -= A(m x k) * B(k x n).
//
// This is the UPDATE-phase DGEMM (the rank-NB update of the trailing matrix,
// Sec. I / Sec. II), where nearly all of the flops of the method are spent.
// At NB = 512 its arithmetic intensity is NB/8 = 64 flop per byte of C
// traffic, far above the MI355X ridge (78.6 TFLOP/s / 8 TB/s ~ 9.8), so the
// kernel is bound by the FP64 matrix cores.
//
// Two kernels (both FP64 MFMA, accumulators in AGPRs, XCD-aware tile order):
//  * gemm_stream_kernel -- the hot one, used wherever its preconditions hold
//    (the whole trailing update at the benchmark's sizes): v_mfma_f64_16x16x4,
//    operands moved global -> LDS by DMA; described where it is defined.
//  * gemm_sub_kernel -- the fallback for any shape and alignment:
//    v_mfma_f64_4x4x4_4b, register-staged double-buffered LDS.
// With accumulators in AGPRs both MFMA forms sustain ~72 TFLOP/s in a pure
// issue loop on gfx950 (with accumulators in ordinary VGPRs the 16x16x4 form
// drops to ~48, because its C operand then shares the register read ports
// with A and B).
//
// gemm_sub_kernel in detail
//  * The instruction holds 4 independent blocks b: lane 16k+4b+i supplies
//    A_b(i,k), lane 16k+4b+j supplies B_b(k,j), and lane 16i+4b+j holds
//    D_b(i,j) (layout checked on the hardware).  All four blocks get the same
//    4-row slice of A (the A value depends only on lane%4 and lane/16) and
//    consecutive 4-column slices of B, so one instruction updates a 4 x 16
//    strip: lane d holds C(4I + d/16, 16G + d%16) for row group I, column
//    group G.
//  * Block tile BM x BN, K staged BK = 16 at a time through double-buffered
//    LDS (one barrier per stage); each wave owns a (BM/WM) x (BN/WN) sub-tile
//    of accumulators that stay in registers for the whole K loop.
//  * Accumulators start from zero; the epilogue applies C <- C - acc a
//    column group at a time.  Every element is therefore C - sum_k a_ik b_kj
//    with the same k order and the same instruction whatever the tiling --
//    the look-ahead split of the update reproduces the unsplit update bit for
//    bit.
//  * Workgroups are dispatched round-robin over the 8 XCDs (each with its own
//    L2).  The block index is remapped so that each XCD receives a contiguous
//    run of tiles, and tiles are ordered in groups of kGroupM tile-rows so the
//    workgroups resident on one XCD share A row-panels and B column-panels in
//    that XCD's L2.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int BK = 16;
constexpr int kGroupM = 4;  // measured best of 1, 2, 4, 8, 16, 32 at N = 163840 (4 over 8: +0.7-1.2 %)

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
    tile_of_block(blockIdx.x, (int64_t)gridDim.x, tiles_m, tiles_n, kGroupM, tm, tn);
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

// ---------------------------------------------------------------------------
// Streamed kernel: v_mfma_f64_16x16x4_f64, operands moved global -> LDS by
// DMA, fragments read one k-step ahead.
//
//  * Tile 128 x BN (BN = 128 or 64), 4 waves (2 x 2), each a 64 x BN/2
//    sub-tile of 16 x 16 blocks.  K is staged 16 at a time in double-buffered
//    LDS.  Every wave moves its share of the next stage with
//    global_load_lds_dwordx4 (64 lanes x 16 bytes straight into 1 KB of LDS,
//    no staging registers): A as whole 128-row columns, B as chunks of 8
//    columns x 16 k.  These loads are issued from inline assembly: the
//    compiler would otherwise wait for them before every LDS read, since it
//    cannot tell the two buffers apart.  The kernel waits for them itself
//    (s_waitcnt vmcnt(0)) before the barrier that publishes a stage.
//  * B sits in LDS as [column][k] with an XOR swizzle on the k pairs (slot s
//    of column c holds pair s ^ ((c >> 1) & 7)); A as [k][row] padded to 144
//    rows.  The fragment reads of 16 lanes x 4 k are then free of bank
//    conflicts.
//  * The MFMA is issued with B's fragment as the first operand, which
//    computes the transposed block: lane l ends up holding C(16i + l%16,
//    16g + 4r + l/16) in register r, i.e. 16 consecutive rows of 4 columns per
//    store instruction (4 full cache lines instead of 16 partial ones).  The
//    products and their k order are those of the untransposed form.
//  * Accumulators start at zero and the epilogue applies C <- C - acc, so
//    each element is C - sum_k a_ik b_kj in the same order whatever the
//    tiling or the column split of the update.
//  * Requirements (checked by the launcher, which otherwise uses
//    gemm_sub_kernel): k a multiple of 32, m even, lda and ldb even, A and B
//    16-byte aligned, ldb < 2^22.  Ragged m and n are handled by clamping the
//    rows and columns the DMA reads and masking the epilogue.
// ---------------------------------------------------------------------------
constexpr int SBM = 128;         // tile rows
constexpr int SBK = 16;          // k per LDS stage
constexpr int SAS = SBM + 16;    // LDS row pitch of A (doubles): k rows 128 bytes apart modulo 256

#define HPLX_LDS(p) ((__attribute__((address_space(3))) void *)(p))

template <int BN, int OCC, int TRAIL>
__global__ __launch_bounds__(256, OCC) void gemm_stream_kernel(
    int64_t m, int64_t n, int64_t k, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double *__restrict__ C, int64_t ldc, int64_t tiles_m,
    int64_t tiles_n)
{
    constexpr int NW = 4, WM = 2, WN = 2;
    constexpr int TM = SBM / WM, TN = BN / WN, FR = TM / 16, FC = TN / 16;
    constexpr int A_INST = SBK / NW;     // A columns per wave per stage
    constexpr int B_INST = BN / 8 / NW;  // 8-column B chunks per wave per stage
    static_assert(A_INST * NW == SBK && B_INST * NW * 8 == BN && FC >= 1, "DMA split");
    asm volatile("" ::: "a0");  // accumulators in AGPRs (see gemm_sub_kernel)
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) double As[2][SBK][SAS];
    __shared__ __attribute__((aligned(16))) double Bs[2][BN][SBK];

    int64_t tm, tn;
    tile_of_block(blockIdx.x, (int64_t)gridDim.x, tiles_m, tiles_n, kGroupM, tm, tn);
    const int64_t m0 = tm * SBM, n0 = tn * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & (NW - 1);
    const int wm = wave % WM, wn = wave / WM;

    // DMA sources.  A: lane l moves rows 2l, 2l+1 of a column (past the last
    // row: the last pair, whose values are never stored).  B: lane l of chunk
    // c8 moves the k pair (l%8) ^ h of column 8*c8 + l/8 (past the last
    // column: column n-1), h = ((8*c8 + l/8) >> 1) & 7.
    const int64_t a_pair = (2 * lane < m - m0 - 1) ? 2 * lane : (m - m0 - 2);
    const uint32_t a_lane = 8u * (uint32_t)a_pair;
    const char *a_tile = (const char *)(A + m0);
    const char *b_tile = (const char *)(B + (size_t)n0 * (size_t)ldb);
    uint32_t b_lane[B_INST];
#pragma unroll
    for (int q = 0; q < B_INST; ++q) {
        const int col = 8 * (wave * B_INST + q) + (lane >> 3);
        const int h = (col >> 1) & 7;
        const int64_t colc = (col < n - n0) ? col : (n - n0 - 1);
        b_lane[q] = (uint32_t)colc * (uint32_t)ldb * 8u + 16u * (uint32_t)((lane & 7) ^ h);
    }
    const uint32_t lds_a = (uint32_t)(uintptr_t)HPLX_LDS(&As[0][0][0]);
    const uint32_t lds_b = (uint32_t)(uintptr_t)HPLX_LDS(&Bs[0][0][0]);
    auto dma_stage = [&](int s, int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < A_INST; ++q) {
            const char *src = a_tile + (size_t)(s * SBK + wave * A_INST + q) * (size_t)lda * 8;
            const uint32_t dst = lds_a + 8u * (uint32_t)((buf * SBK + wave * A_INST + q) * SAS);
            asm volatile("global_load_lds_dwordx4 %0, %1" ::"v"(a_lane), "s"(src), "{m0}"(dst) : "memory");
        }
#pragma unroll
        for (int q = 0; q < B_INST; ++q) {
            const char *src = b_tile + (size_t)(s * SBK) * 8;
            const uint32_t dst = lds_b + 8u * (uint32_t)((buf * BN + 8 * (wave * B_INST + q)) * SBK);
            asm volatile("global_load_lds_dwordx4 %0, %1" ::"v"(b_lane[q]), "s"(src), "{m0}"(dst) : "memory");
        }
    };
    auto dma_wait = [&]() __attribute__((always_inline)) { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); };

    d4 acc[FR][FC];
#pragma unroll
    for (int i = 0; i < FR; ++i)
#pragma unroll
        for (int g = 0; g < FC; ++g) acc[i][g] = (d4){0.0, 0.0, 0.0, 0.0};

    // fragments: A(16i + l%16, 4*k4 + l/16) and B(4*k4 + l/16, 16g + l%16) of the wave's sub-tile
    const int kq = lane >> 4;
    const double *pa_l = &As[0][kq][wm * TM + (lane & 15)];
    const int h2 = 2 * ((lane & 15) >> 1);
    const double *pb_l[4];
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) pb_l[k4] = &Bs[0][wn * TN + (lane & 15)][(4 * k4 + kq) ^ h2];
    auto rd_a = [&](int buf, int k4, int i) __attribute__((always_inline)) -> double {
        return pa_l[buf * SBK * SAS + 4 * k4 * SAS + 16 * i];
    };
    auto rd_b = [&](int buf, int k4, int g) __attribute__((always_inline)) -> double {
        return pb_l[k4][buf * BN * SBK + 16 * g * SBK];
    };
    double af[FR], b0[FC], b1[FC];

    // One k-step: MFMAs on (af, bc); the next step's fragments, at (nbuf, nk4),
    // are read as the current ones die.
    auto step = [&](double(&bc)[FC], double(&bn)[FC], int nbuf, int nk4, bool has_next) __attribute__((always_inline)) {
        if (has_next) {
#pragma unroll
            for (int g = 0; g < FC; ++g) bn[g] = rd_b(nbuf, nk4, g);
        }
#pragma unroll
        for (int i = 0; i < FR; ++i) {
#pragma unroll
            for (int g = 0; g < FC; ++g) acc[i][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(bc[g], af[i], acc[i][g], 0, 0, 0);
            if (has_next) af[i] = rd_a(nbuf, nk4, i);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // Stage s (in buffer buf): the DMA of stage s+1 into the other buffer is in
    // flight during its first three k-steps; the fourth runs after the barrier
    // that publishes stage s+1, reading that stage's first fragments.
    auto stage = [&](int s, int buf, bool more) __attribute__((always_inline)) {
        if (more) dma_stage(s + 1, buf ^ 1);
        step(b0, b1, buf, 1, true);
        step(b1, b0, buf, 2, true);
        step(b0, b1, buf, 3, true);
        if (more) {
            dma_wait();
            __syncthreads();
            step(b1, b0, buf ^ 1, 0, true);
        } else {
            step(b1, b0, buf, 0, false);
        }
    };

    const int nst = (int)(k / SBK);  // even
    dma_stage(0, 0);
    dma_wait();
    __syncthreads();
#pragma unroll
    for (int g = 0; g < FC; ++g) b0[g] = rd_b(0, 0, g);
#pragma unroll
    for (int i = 0; i < FR; ++i) af[i] = rd_a(0, 0, i);
    int s = 0;
    for (; s + 2 < nst; s += 2) {
        stage(s, 0, true);
        stage(s + 1, 1, true);
    }
    stage(s, 0, true);
    stage(s + 1, 1, false);

    // epilogue: acc[i][g][r] belongs to C(row + 16i, col + 16g + 4r)
    const int64_t row = m0 + wm * TM + (lane & 15);
    const int64_t col = n0 + wn * TN + (lane >> 4);
    double *pc = C + off(row, col, ldc);
    if (m0 + SBM <= m && n0 + BN <= n) {
#pragma unroll
        for (int g = 0; g < FC; ++g) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double *pcol = pc + (size_t)(16 * g + 4 * r) * (size_t)ldc;
#pragma unroll
                for (int i = 0; i < FR; ++i) pcol[16 * i] = pcol[16 * i] - acc[i][g][r];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int g = 0; g < FC; ++g) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (col + 16 * g + 4 * r >= n) continue;
                double *pcol = pc + (size_t)(16 * g + 4 * r) * (size_t)ldc;
#pragma unroll
                for (int i = 0; i < FR; ++i)
                    if (row + 16 * i < m) pcol[16 * i] = pcol[16 * i] - acc[i][g][r];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int BN, int OCC, int TRAIL>
int launch_stream(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                  double *C, int64_t ldc, hipStream_t st)
{
    const int64_t tiles_m = (m + SBM - 1) / SBM, tiles_n = (n + BN - 1) / BN;
    const int64_t nwg = tiles_m * tiles_n;
    if (nwg > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL((gemm_stream_kernel<BN, OCC, TRAIL>), dim3((unsigned)nwg), dim3(256), 0, st, m, n, k, A, lda,
                       B, ldb, C, ldc, tiles_m, tiles_n);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

// Whether gemm_stream_kernel can run this product.  Depends only on m, k, the
// leading dimensions and the operand alignment -- not on n -- so the column
// pieces of one update all take the same kernel family.
bool stream_ok(int64_t m, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb)
{
    return k >= 32 && k % 32 == 0 && m >= 2 && m % 2 == 0 && lda % 2 == 0 && ldb % 2 == 0 &&
           ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0 && ldb < ((int64_t)1 << 22);
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

// variant: 0 = auto; 1 = 128x128, 2 = 128x64, 3 = 64x64, 4 = 128x32 (gemm_sub_kernel);
// 5 = 128x128, 6 = 128x64 (gemm_stream_kernel, where stream_ok holds, else auto).
// The caller adds kGemmTrailing for the trailing update.
int launch_gemm_sub(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                    int64_t ldb, double *C, int64_t ldc, int variant, hipStream_t st)
{
    if (m <= 0 || n <= 0 || k <= 0) return HPL_OK;
    const bool trail = (variant & kGemmTrailing) != 0;
    variant &= ~kGemmTrailing;
    const bool stream = stream_ok(m, k, A, lda, B, ldb);
    if ((variant == 5 || variant == 6) && !stream) variant = 0;
    if (variant == 0) {
        if (stream)
            variant = (n <= 64 || ((m + 127) / 128) * ((n + 127) / 128) < 512) ? 6 : 5;
        else if (n <= 32)
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
        case 5: return launch_stream<128, 2, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        case 6: return launch_stream<64, 3, 1>(m, n, k, A, lda, B, ldb, C, ldc, st);
        default: return HPL_ERR_INTERNAL;
        }
    }
    switch (variant) {
    case 1: return launch_cfg<128, 128, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 2: return launch_cfg<128, 64, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 3: return launch_cfg<64, 64, 2, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 4: return launch_cfg<128, 32, 4, 1, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 5: return launch_stream<128, 2, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    case 6: return launch_stream<64, 3, 0>(m, n, k, A, lda, B, ldb, C, ldc, st);
    default: return HPL_ERR_INTERNAL;
    }
}

}  // namespace hplx
