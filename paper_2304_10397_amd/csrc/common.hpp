// common.hpp -- internal declarations shared by the libhplx translation units.
//
// Every kernel here is written for gfx950 (CDNA4): 64-wide wavefronts, FP64
// MFMA (v_mfma_f64_16x16x4_f64), 160 KB of LDS per CU.  Matrices are FP64,
// column-major, 64-bit offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hpl.h"

namespace hplx {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// 64-bit element offset of (i, j) in a column-major matrix.
__host__ __device__ __forceinline__ size_t off(int64_t i, int64_t j, int64_t ld)
{
    return (size_t)i + (size_t)j * (size_t)ld;
}

// p[0] when ok, else z, with the load issued unconditionally (from p, or from
// the always-valid address safe): a guarded load written as "ok ? p[0] : z"
// is compiled to a branch around the load followed by a wait for it, so a
// run of such loads costs one memory round trip each; these do not.
template <typename T>
__device__ __forceinline__ T load_or(bool ok, const T *p, const T *safe, T z)
{
    const T v = *(ok ? p : safe);
    return ok ? v : z;
}

// Block index -> output tile (tm, tn) of a tiles_m x tiles_n grid.  Workgroups
// are dispatched round-robin over the 8 XCDs, each with its own L2: the index
// is remapped so that each XCD receives a contiguous run of tiles, and the run
// is ordered in groups of group_m tile-rows (column-major inside a group), so
// that the workgroups resident on one XCD share A row-panels and B
// column-panels in that XCD's L2.
__device__ __forceinline__ void tile_of_block(int64_t bid, int64_t nwg, int64_t tiles_m, int64_t tiles_n,
                                              int64_t group_m, int64_t &tm, int64_t &tn)
{
    const int64_t xcd = bid & 7, in_xcd = bid >> 3;
    const int64_t per = nwg >> 3, rem = nwg & 7;
    const int64_t lin = xcd * per + (xcd < rem ? xcd : rem) + in_xcd;
    const int64_t group_size = group_m * tiles_n;
    const int64_t g = lin / group_size;
    const int64_t first_m = g * group_m;
    const int64_t gm = (tiles_m - first_m) < group_m ? (tiles_m - first_m) : group_m;
    const int64_t r = lin - g * group_size;
    tm = first_m + r % gm;
    tn = r / gm;
}

// Value of v held by lane l of the wave (l uniform across the wave): two
// v_readlane_b32, a few cycles, instead of an LDS round trip.
__device__ __forceinline__ double read_lane(double v, int l)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Wave-wide reductions returned to every lane: rotations within each row of 16
// lanes through DPP (no LDS traffic), then the four row results read out and
// combined.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double wave_max(double x)
{
    x = fmax(x, dpp_mov<0x128>(x));  // row_ror:8
    x = fmax(x, dpp_mov<0x124>(x));  // row_ror:4
    x = fmax(x, dpp_mov<0x122>(x));  // row_ror:2
    x = fmax(x, dpp_mov<0x121>(x));  // row_ror:1
    return fmax(fmax(read_lane(x, 0), read_lane(x, 16)), fmax(read_lane(x, 32), read_lane(x, 48)));
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned x)
{
    x = min(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xf, 0xf, false));
    x = min(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x124, 0xf, 0xf, false));
    x = min(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x122, 0xf, 0xf, false));
    x = min(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x121, 0xf, 0xf, false));
    const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)x, 0), b = (unsigned)__builtin_amdgcn_readlane((int)x, 16);
    const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)x, 32), d = (unsigned)__builtin_amdgcn_readlane((int)x, 48);
    return min(min(a, b), min(c, d));
}

// ---------------------------------------------------------------------------
// Error plumbing (host).
// ---------------------------------------------------------------------------
void note_hip_error(hipError_t e, const char *what, const char *file, int line);
void note_error(const char *what, const char *file, int line);

#define HPLX_TRY(call)                                                         \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ::hplx::note_hip_error(e_, #call, __FILE__, __LINE__);             \
            return HPL_ERR_HIP;                                                \
        }                                                                      \
    } while (0)

#define HPLX_TRY_LAUNCH()  HPLX_TRY(hipGetLastError())

#define HPLX_PROPAGATE(expr)                                                   \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_ != HPL_OK) return rc_;                                         \
    } while (0)

// ---------------------------------------------------------------------------
// Random input generator: counter-based SplitMix64 (Steele, Lea, Flood 2014).
// ---------------------------------------------------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kStreamStride = 0xD1B54A32D192ED03ull;

__host__ __device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// SplitMix64 state of (seed, stream): first output of state seed + stream*stride.
__host__ __device__ __forceinline__ uint64_t stream_state(uint64_t seed, uint64_t stream)
{
    return sm64_mix(seed + stream * kStreamStride + kGamma);
}

// Value at linear index idx: idx-th SplitMix64 output, top 53 bits -> [-0.5, 0.5).
__host__ __device__ __forceinline__ double gen_value(uint64_t s0, uint64_t idx)
{
    uint64_t h = sm64_mix(s0 + (idx + 1ull) * kGamma);
    return (double)(h >> 11) * 0x1.0p-53 - 0.5;
}

// ---------------------------------------------------------------------------
// Kernel launchers (each returns HPL_OK or an HPL_ERR_* after noting the cause).
// ---------------------------------------------------------------------------

// gen.hip
int launch_generate(uint64_t s0, double *M, int64_t rows, int64_t cols, int64_t ld,
                    hipStream_t st);
// Residual partials: result slots (uint64 bit patterns of non-negative doubles,
// combined with atomicMax): red[0] = ||A||inf, then per rhs c: red[1+3c+0] =
// ||r_c||inf, red[1+3c+1] = ||x_c||inf, red[1+3c+2] = ||b_c||inf.  red must be
// zeroed first.
int launch_residual(const double *A, int64_t lda, bool gen, uint64_t s0, int64_t n,
                    const double *X, int64_t ldx, const double *B, int64_t ldb, int64_t nrhs,
                    unsigned long long *red, hipStream_t st);
int launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long v, hipStream_t st);
// the paper's CPU FACT (host memory, T threads)
constexpr int kHostPanelMaxThreads = 256;
int host_panel_factor(double *P, int64_t m, int64_t nb, int64_t ld, int32_t *ipiv, int threads, int64_t *info);

// batched small systems (one persistent launch)
constexpr int kBatchMaxN = 512;
constexpr int kBatchMaxRhs = 16;
constexpr int kBatchBuckets = kBatchMaxN / 32;  // size buckets (n - 1) / 32 of the tuned table
constexpr uint64_t kBatchSizeStream = 3;  // generator stream of the batch's sizes
// occ: workgroups (systems in flight) per CU, 1 or 2; vtab: the variant
// (HPL_BATCH_VARIANTS of them) of each size bucket; cus: compute units.
int launch_batched_solve(int64_t count, const int32_t *sizes, const int64_t *aoff, const int64_t *voff,
                         const int32_t *order, double *A, int32_t *ipiv, double *B, const double *W, double *GB,
                         double *GA, int nrhs, int mode, int64_t *info, unsigned *counter, int occ,
                         const signed char *vtab, int cus, hipStream_t st);

// gemm.hip: C(m x n) -= A(m x k) * B(k x n).  variant: 0 auto, 1..4 tile shape;
// OR kGemmTrailing for the trailing update (a separately named instance).
constexpr int kGemmTrailing = 0x100;
int launch_gemm_sub(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc, int variant,
                    hipStream_t st);

// skinny.hip: C(m x n) -= A(m x k) * B(k x n) for k = 16, 32 or 64 and n <= k
// (the updates inside the recursive panel).
bool gemm_skinny_ok(int64_t n, int64_t k);
int launch_gemm_skinny(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B, int64_t ldb,
                       double *C, int64_t ldc, hipStream_t st);

// trsm.hip: B(nbk x ncols) <- L^{-1} B, L unit lower nbk x nbk (nbk <= 512).
int launch_trsm_llnu(const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nbk,
                     int64_t ncols, hipStream_t st);
// The same small solve (one wave per column) for the FP32 panel of the
// mixed-precision factorization: nbk <= 512, ncols <= 4096.
bool trsm32_small_ok(int64_t nbk, int64_t ncols);
int launch_trsm32_small(const float *L, int64_t ldl, float *B, int64_t ldb, int64_t nbk, int64_t ncols,
                        hipStream_t st, unsigned *mx = nullptr);

// laswp.hip
// Interchanges k = 0..cnt-1: row r0+k <-> ipiv[k] (global rows, ipiv[k] >= r0+k),
// cnt <= kMaxSwaps, composed into a permutation of the touched rows.  Output
// "slot list": nslots, rows[s] (global rows), srcslot[s]: after the
// interchanges, row rows[s] holds what row rows[srcslot[s]] held before.
constexpr int kMaxSwaps = 512;
struct SwapPlan {
    int32_t *rows;     // [2*kMaxSwaps]
    int32_t *srcslot;  // [2*kMaxSwaps]
    int32_t *nslots;   // [1]
    int *err;          // set to 1 (never cleared by the kernel) if a pivot lies outside [r0+k, nrows)
};
int launch_swap_plan(const int32_t *ipiv, int cnt, int64_t r0, int64_t nrows, bool reverse, SwapPlan plan,
                     hipStream_t st);
// Plans of all kMaxSwaps-sized chunks of ipiv[0..total) at once (chunk q covers
// rows r0 + q*kMaxSwaps ...), laid out with stride kPlanStride int32 per chunk:
// rows at [0, 2*kMaxSwaps), srcslot at [2*kMaxSwaps, 4*kMaxSwaps), nslots at 4*kMaxSwaps.
constexpr int kPlanStride = 4 * kMaxSwaps + 64;
int launch_swap_plans_all(const int32_t *ipiv, int64_t total, int64_t r0, int64_t nrows, bool reverse,
                          int32_t *plans, int *err, hipStream_t st);
// Applies a plan to columns [col0, col0+ncols) of A.
int launch_laswp(double *A, int64_t lda, int64_t col0, int64_t ncols, SwapPlan plan, int64_t max_wgs,
                 hipStream_t st);

// panel.hip: leaf of the recursive panel factorization.
struct LeafSync {
    unsigned long long *counter;  // monotonic barrier counter
    int *abort_flag;              // set on barrier time-out
    double *slots;                // [2][kLeafMaxWGs][kLeafSlot]
    double *top;                  // [2][kLeafMaxW]
    unsigned long long *info;     // min over singular columns of (global col + 1)
    unsigned long long *tslots;   // tagged words of the register leaf: [2][kLeafMaxWGs][kLeafSlotWords]
    unsigned long long *ttop;     // tagged diagonal row: [2][64]
};
constexpr int kLeafMaxW = 64;
constexpr int kLeafMaxWGs = 256;
constexpr int kLeafSlot = kLeafMaxW + 2;
constexpr int kLeafSlotWords = 2 * 32 + 3 + 5;  // tagged words per slot of the register leaf (72)
int launch_panel_leaf(double *A, int64_t lda, int64_t c, int64_t m, int w, int32_t *ipiv,
                      LeafSync sync, unsigned long long bar_base, int G, hipStream_t st);
// Number of workgroups the leaf kernel uses for m rows, width w, limit gmax.
int leaf_groups(int64_t m, int w, int gmax);
// Register-resident leaf (w <= 32, at most 1024 rows per workgroup): number of
// workgroups for m rows, or 0 if it does not apply.  The launch also runs the
// in-leaf interchanges of the finished L columns.  tag0 must differ from every
// tag used before (tags tag0+1 .. tag0+w are consumed).
int leaf_reg_groups(int64_t m, int w);
int launch_leaf_reg(double *A, int64_t lda, int64_t c, int64_t m, int w, int32_t *ipiv, LeafSync sync,
                    uint32_t tag0, int G, hipStream_t st);

// solve.hip
// One diagonal block [r0, r0+bs) (bs <= 64, nrhs <= 64): finish it, then update
// rows [row_begin, row_end).  mode: 0 = L unit lower (forward), 1 = U upper
// (backward), 2 = U^T (forward), 3 = L^T unit (backward).  done: a device word
// that is zero between launches (the launch counts its workgroups on it and
// leaves it at zero); launches that share it must not overlap in time.
int launch_solve_block(const double *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs,
                       int64_t r0, int64_t bs, int64_t row_begin, int64_t row_end, int mode,
                       unsigned *done, hipStream_t st);
// Applies nchunks plans (kPlanStride layout) to B in order, or in reverse order.
int launch_apply_plans_seq(double *B, int64_t ldb, int64_t nrhs, const int32_t *plans,
                           int64_t nchunks, bool reverse, hipStream_t st);
// The whole solve of A X = B (trans 0) or A^T X = B (trans 1) with the factors
// LU and ipiv, on stream st.  plans: ceil(n/kMaxSwaps) * kPlanStride int32;
// pivot_err: raised (never cleared) on a pivot outside [k, n); done: a zero
// word (the block launches leave it at zero).
int solve_sequence(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n, int64_t lda,
                   int64_t ldb, int trans, int32_t *plans, int *pivot_err, unsigned *done, hipStream_t st);
int solve_upper_sequence(const double *U, double *B, int64_t nrhs, int64_t n, int64_t lda, int64_t ldb, unsigned *done,
                         hipStream_t st);

// Pure FP64 MFMA issue loop (probe.hip): nwg workgroups of 256 threads, iters
// rounds of 16 independent 16x16x4 MFMAs per wave; mfma_peak_flops is its flop count.
// iters must be a multiple of the loop's unroll; mfma_peak_rounds rounds it up.
int launch_mfma_peak(double *out, int64_t nwg, int64_t iters, hipStream_t st);
int64_t mfma_peak_rounds(int64_t iters);
double mfma_peak_flops(int64_t nwg, int64_t iters);

// Differentiable solve (gen.hip, grad.hip): Box-Muller normal generator, M(i,i) += alpha,
// and D = -G X^T for n x k panels G, X (rank-k outer product written once).
int launch_generate_normal(uint64_t s0, double *M, int64_t rows, int64_t cols, int64_t ld, hipStream_t st);
int launch_add_diagonal(double *M, int64_t n, int64_t ld, double alpha, hipStream_t st);
int launch_grad_a(const double *G, int64_t ldg, const double *X, int64_t ldx, int64_t n, int64_t k, double *D,
                  int64_t ldd, hipStream_t st);

// Mixed-precision LU and refinement (mxp.hip); solve_block with FP32 factors (solve.hip).
int launch_mxp_diag(double *A, int64_t n, int64_t lda, hipStream_t st);
int launch_cvt_f64_f32(const double *A, int64_t lda, float *B, int64_t ldb, int64_t rows, int64_t cols,
                       hipStream_t st);
// widest FP32 panel leaf and triangular-solve leaf (one launch each)
constexpr int kPanel32LeafMax = 64, kTrsm32LeafMax = 64;
// With mx, the FP32 leaves fold the largest |value| they store into *mx (the
// panel leaf: rows from l21_row0 on, i.e. L21; the solve leaves: all of it).
int launch_panel32_leaf(float *A, int64_t lda, int64_t c, int64_t n, int w, unsigned long long *info,
                        unsigned *done, hipStream_t st, unsigned *mx = nullptr, int64_t l21_row0 = 0);
int launch_trsm32_leaf(const float *L, int64_t ldl, float *B, int64_t ldb, int nbk, int64_t ncols, hipStream_t st,
                       unsigned *mx = nullptr);
int launch_sgemm32(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                   float *C, int64_t ldc, hipStream_t st);
// -L21 and U12 scaled (the exponent from mx) and rounded into the blocked
// low-precision layout (1 KB blocks of 16 rows x 32 k, ordered by k slab then
// 16-row group; sa, sb = slab strides in elements, multiples of 512; A16 and
// B16 point at the block of the first row and k); reset[0..1] cleared.
int launch_mxp_convert(int fmt, const float *L, int64_t ldl, int64_t m, const float *U, int64_t ldu, int64_t ncols,
                       int w, const unsigned *mx, unsigned *reset, void *A16, int64_t sa, void *B16, int64_t sb,
                       hipStream_t st);
int launch_hgemm_update(int fmt, int64_t m, int64_t n, int64_t K, const void *A16, int64_t sa, const void *B16,
                        int64_t sb, float *C, int64_t ldc, hipStream_t st);
// r = b - A x with kResSplit column chunks; part holds 2 kResSplit n doubles of partial sums.
constexpr int kResSplit = 16;
int launch_mxp_residual(const double *A, int64_t lda, const double *x, const double *b, double *r, int64_t n,
                        bool anorm, double *part, unsigned long long *red, hipStream_t st);
int launch_axpy(double *x, const double *d, int64_t n, hipStream_t st);
int launch_solve_block_f32(const float *T, int64_t ldt, double *B, int64_t ldb, int64_t nrhs, int64_t r0, int64_t bs,
                           int64_t row_begin, int64_t row_end, int mode, unsigned *done, hipStream_t st);

}  // namespace hplx
