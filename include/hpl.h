/*
 * hpl.h -- C ABI of libhplx: the High-Performance Linpack hot path on one
 * AMD Instinct MI355X (gfx950).
 *
 * The method (Chalmers, Kurzak, McDougall, Bauman, "Optimizing
 * High-Performance Linpack for Exascale Accelerated Architectures"):
 * a random dense N x N double-precision system A x = b is solved by blocked
 * Gaussian elimination with partial pivoting (Sec. I, Sec. II).  Each
 * iteration along the diagonal factors an NB-column panel with pivoting
 * inside the panel (FACT), applies the panel's NB interchanges to the rest of
 * the matrix (RS), solves for the U block row with the unit-lower diagonal
 * block (DTRSM) and applies the rank-NB update to the trailing matrix (DGEMM)
 * (Sec. I bullets, Sec. II).  A look-ahead updates the next panel's columns
 * first so that the next FACT overlaps the rest of the update (Sec. III).
 * With A = P L U, A x = b becomes U x = L^{-1} P^{-1} b, solved by applying
 * U^{-1} (Sec. II).
 *
 * Conventions shared by every entry point
 *   - All matrices are FP64, column-major: element (i, j) of a matrix with
 *     leading dimension ld is at ptr[i + j*ld].  Sizes and leading dimensions
 *     are int64_t; offsets are computed in 64 bits (N^2 exceeds 2^31).
 *   - Matrix and pivot pointers are DEVICE pointers, allocated and owned by
 *     the caller.  Output arrays documented as host arrays (info, out) are
 *     host pointers.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  Work is ordered
 *     on that stream; the library may use internal streams for the
 *     look-ahead and joins them back before returning.  Every entry point
 *     returns after its work on the device has completed.
 *   - Return value: 0 on success; -k if argument k (1-based) is invalid,
 *     detected on the host before any HIP call; a positive HPL_ERR_* code on a
 *     runtime failure (hpl_strerror gives text, hpl_last_error_detail the
 *     failing call).  Nothing is modified when -k is returned.
 *   - The library allocates only workspace (never O(n^2)), once per device,
 *     lazily on first use; hpl_release frees it.  Calls on one device must not
 *     overlap in time (the workspace is shared); the library is not
 *     re-entrant per device.
 *   - The library loads on a machine without a GPU; argument validation and
 *     hpl_strerror / hpl_set_option / hpl_get_option work there.
 */
#ifndef HPLX_HPL_H
#define HPLX_HPL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hpl_status {
    HPL_OK = 0,
    HPL_ERR_HIP = 1,      /* a HIP runtime call failed (see hpl_last_error_detail) */
    HPL_ERR_NOMEM = 2,    /* workspace allocation failed */
    HPL_ERR_DEVICE = 3,   /* no device, or the current device is not gfx950 */
    HPL_ERR_INTERNAL = 4  /* a kernel reported failure (e.g. panel barrier time-out) */
};

/*
 * hpl_factor -- LU factorization with partial pivoting, P A = L U
 * (Sec. I FACT/RS/UPDATE, Sec. II, Sec. III look-ahead).
 *   1 A     device, n x n at leading dimension lda; overwritten by L (unit
 *           diagonal not stored) below the diagonal and U on and above it.
 *   2 n     order, 0 <= n <= 2^31 - 1 (n = 0 returns at once).
 *   3 lda   leading dimension, lda >= max(1, n).
 *   4 nb    block size (panel width), 1 <= nb <= 1024.
 *   5 ipiv  device int32[n]: 0-based, row k was interchanged with row
 *           ipiv[k] >= k, interchanges applied in the order k = 0..n-1 and
 *           across all n columns (LAPACK getrf form: P = S_{n-1}...S_0).
 *   6 info  host int64*: 0, or k + 1 for the first k with U(k,k) exactly 0 (the
 *           pivot column was all zero); the factorization still completes and
 *           that column is left unscaled.
 *   7 hip_stream
 * The pivot is the row of largest |a| in the column, the lowest row index on
 * ties, so results do not depend on the reduction order.  Look-ahead on or
 * off (hpl_set_option) gives bit-identical results.
 */
int hpl_factor(double *A, int64_t n, int64_t lda, int64_t nb, int32_t *ipiv, int64_t *info,
               void *hip_stream);

/*
 * hpl_solve -- solve with the factors of hpl_factor (Sec. II: apply P, then
 * L^{-1}, then U^{-1}).
 *   1 LU    device, n x n at lda, as returned by hpl_factor (not modified).
 *   2 ipiv  device int32[n] from hpl_factor.
 *   3 B     device, n x nrhs at ldb; overwritten by the solution X.
 *   4 nrhs  number of right-hand sides, >= 0.
 *   5 n     order, >= 0.
 *   6 lda   >= max(1, n).
 *   7 ldb   >= max(1, n).
 *   8 trans 0: A X = B.  1: A^T X = B (U^T forward, L^T backward, then the
 *           interchanges in reverse order).
 *   9 hip_stream
 * LU and B must not overlap.  A zero diagonal of U yields inf/NaN in X (no
 * check), as the factorization's info reported.
 */
int hpl_solve(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n,
              int64_t lda, int64_t ldb, int trans, void *hip_stream);

/*
 * hpl_solve_augmented -- the HPL benchmark's own formulation (Sec. II): A x = b
 * is treated as the augmented system [A | B], which the blocked LU with
 * partial pivoting turns into U X = L^{-1} P^{-1} B; X then follows by back
 * substitution.  The row interchanges of each panel (the RS phase, Sec. II)
 * reach only the columns to the right of the panel -- the remaining matrix and
 * the right-hand sides -- never the finished L columns to its left.
 *   1 A     device, n x (n + nrhs) at leading dimension lda: columns [0, n)
 *           the matrix, columns [n, n + nrhs) the right-hand sides B.  On
 *           return U is on and above the diagonal; below it, the multipliers of
 *           each nb-column panel in the row order of that panel's own
 *           factorization (the interchanges of later panels not applied to
 *           them, unlike hpl_factor's LAPACK form); columns [n, n + nrhs) hold
 *           the solution X (when info = 0).
 *   2 n     order, 0 <= n <= 2^31 - 1.
 *   3 lda   >= max(1, n).
 *   4 nb    panel width, 1 <= nb <= 1024.
 *   5 nrhs  right-hand sides, >= 0.
 *   6 ipiv  device int32[n]: as hpl_factor's (the same pivots).
 *   7 info  host int64*: as hpl_factor's; when info > 0 the back substitution
 *           is skipped and columns [n, n + nrhs) hold L^{-1} P^{-1} B.
 *   8 hip_stream
 * The pivots and U are those of hpl_factor on the same matrix; look-ahead on or
 * off gives bit-identical results.  Returns after X is complete.
 */
int hpl_solve_augmented(double *A, int64_t n, int64_t lda, int64_t nb, int64_t nrhs, int32_t *ipiv,
                        int64_t *info, void *hip_stream);

/*
 * hpl_solve_noalloc -- hpl_solve for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments, kernels and results (bit for bit),
 * but its scratch (the interchange plans of ipiv's 512-pivot chunks, a
 * workgroup counter and an error word) lives in a fixed device array inside
 * the library, HPL_SOLVE_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends.  No call allocates: no hipMalloc/hipFree, no events, no
 * library workspace (the first call on a device only looks up the array's
 * device address).
 *   n > HPL_SOLVE_NOALLOC_MAX_N is rejected with -5 before any HIP call
 *   (hpl_last_error_detail names the limit); other arguments as hpl_solve.
 * All calls on one GPU share that GPU's array: calls that overlap in time on
 * one GPU (other streams, other host threads) race.  Each call clears what
 * must start at zero and returns after its work has completed.
 */
#define HPL_SOLVE_NOALLOC_MAX_N 262144
#define HPL_SOLVE_NOALLOC_SCRATCH_BYTES (512 + 4 * 2112 * 512) /* 4.1 MiB */
int hpl_solve_noalloc(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n,
                      int64_t lda, int64_t ldb, int trans, void *hip_stream);

/*
 * hpl_residual -- HPL acceptance test for A X = B with an explicit A.
 *   1 A0 device n x n at lda (the original matrix); 2 n; 3 lda >= max(1,n);
 *   4 X device n x nrhs at ldx; 5 ldx >= max(1,n); 6 B device n x nrhs at ldb;
 *   7 ldb >= max(1,n); 8 nrhs >= 1;
 *   9 out host double[5] = {scaled, ||A X - B||inf, ||A||inf, ||X||inf, ||B||inf},
 *     scaled = ||r||inf / (eps (||A||inf ||x||inf + ||b||inf) n), eps = 2^-53,
 *     computed per column; out[0] is the largest per-column scaled residual
 *     and out[1], out[3], out[4] the largest per-column norms.  The run
 *     passes when out[0] < 16.  NaN anywhere propagates to out[0].
 *  10 hip_stream
 */
int hpl_residual(const double *A0, int64_t n, int64_t lda, const double *X, int64_t ldx,
                 const double *B, int64_t ldb, int64_t nrhs, double *out, void *hip_stream);

/*
 * hpl_residual_gen -- as hpl_residual, with A regenerated on the fly from
 * (seed, stream 0) of hpl_generate instead of being read (at N = 163840 the
 * original A cannot be kept next to its factors).
 *   1 seed; 2 n >= 0; 3 X device; 4 ldx; 5 B device; 6 ldb; 7 nrhs >= 1;
 *   8 out host double[5]; 9 hip_stream.
 */
int hpl_residual_gen(uint64_t seed, int64_t n, const double *X, int64_t ldx, const double *B,
                     int64_t ldb, int64_t nrhs, double *out, void *hip_stream);

/*
 * hpl_generate -- the random system (Sec. II: the benchmark generates a random
 * N x N matrix and right-hand side).  Entries are i.i.d. uniform on
 * [-0.5, 0.5): the value at linear index idx = i + j*rows is the idx-th
 * output of a SplitMix64 sequence (Steele, Lea, Flood, OOPSLA 2014) whose
 * state is the first SplitMix64 output of seed + stream_id * 0xD1B54A32D192ED03,
 * mapped as (h >> 11) * 2^-53 - 0.5 (exact).  Stream 0 is A, stream 1 is b.
 *   1 seed; 2 stream_id; 3 M device rows x cols at ld (written);
 *   4 rows >= 0; 5 cols >= 0; 6 ld >= max(1, rows); 7 hip_stream.
 */
int hpl_generate(uint64_t seed, uint64_t stream_id, double *M, int64_t rows, int64_t cols,
                 int64_t ld, void *hip_stream);

/*
 * Differentiable solve.  For X = A^{-1} B (hpl_factor + hpl_solve) and a loss L
 * with G = dL/dX, the adjoint of the solve is grad_B = A^{-T} G, obtained with
 * hpl_solve(trans = 1) on the saved factors, and grad_A = -grad_B X^T
 * (differentiating A X = B gives A dX = dB - dA X).
 *
 * hpl_solve_grad_a -- dA = -GB X^T, every entry of dA written once.
 *   1 GB   device n x nrhs at ldgb (grad_B);  2 ldgb >= max(1, n)
 *   3 X    device n x nrhs at ldx (the solution);  4 ldx >= max(1, n)
 *   5 n    0 <= n <= 2097120;  6 nrhs >= 0 (nrhs = 0 writes zeros)
 *   7 dA   device n x n at ldda (written, must not overlap GB or X);  8 ldda >= max(1, n)
 *   9 hip_stream
 * Each entry is -(sum over r = 0..nrhs-1 of GB(i,r) X(j,r)), summed in that order.
 */
int hpl_solve_grad_a(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n,
                     int64_t nrhs, double *dA, int64_t ldda, void *hip_stream);

/*
 * hpl_generate_normal -- standard normal values for the loss weights of the
 * differentiable solve: the Box-Muller transform (Box, Muller 1958) of the
 * outputs 2 idx and 2 idx + 1 of the hpl_generate stream (seed, stream_id),
 * u = (h >> 11) 2^-53, z = sqrt(-2 ln(1 - u1)) cos(2 pi u2), idx = i + j*rows.
 * Arguments as hpl_generate.  The values depend on the device's log and cos
 * (within a few units in the last place of a correctly rounded evaluation).
 */
int hpl_generate_normal(uint64_t seed, uint64_t stream_id, double *M, int64_t rows, int64_t cols,
                        int64_t ld, void *hip_stream);

/*
 * hpl_add_diagonal -- M(i,i) += alpha for i < n (the differentiable-solve input
 * A = U[-0.5, 0.5) + 8 I).  1 M device n x n at ld; 2 n >= 0; 3 ld >= max(1, n);
 * 4 alpha; 5 hip_stream.
 */
int hpl_add_diagonal(double *M, int64_t n, int64_t ld, double alpha, void *hip_stream);

/*
 * Mixed precision (HPL-MxP, which the paper mentions alongside HPL, Sec. I):
 * LU in FP16 or BF16 on the matrix cores, then FP64 iterative refinement to
 * the FP64 scaled-residual test.
 *
 * hpl_mxp_generate -- the diagonally dominant input: the hpl_generate matrix
 * of (seed, stream 0), then a_ii = sum_j |a_ij| of the generated row (j in
 * order), so that LU needs no pivoting.
 *   1 seed; 2 A device n x n at lda (written); 3 n >= 0; 4 lda >= max(1, n); 5 hip_stream
 */
int hpl_mxp_generate(uint64_t seed, double *A, int64_t n, int64_t lda, void *hip_stream);

/*
 * hpl_mxp_factor -- LU without pivoting, FP32 storage:
 *   for each NB-column panel: FACT in FP32, U12 = L11^{-1} A12 in FP32, then
 *   A22 += (-L21) U12 with L21 scaled by 2^s and U12 by 2^-s (s on the device
 *   from their maxima: exact, and keeps small multipliers out of FP16's
 *   subnormal range), both rounded to the format, products accumulated in FP32
 *   on v_mfma_f32_16x16x32_{f16,bf16}.
 *   1 A    device FP64 n x n at lda (input, not modified)
 *   2 n    0 <= n < 2^31;  3 lda >= max(1, n)
 *   4 nb   panel width, a multiple of 64 in [64, 4096]
 *   5 fmt  0 = FP16, 1 = BF16
 *   6 LU   device FP32 n x n at ldlu (written: unit-lower L below the
 *          diagonal, U on and above it)
 *   7 ldlu >= max(1, n)
 *   8 info host int64*: 0, or k+1 for the first exactly-zero diagonal of U
 *   9 hip_stream
 * With HPL_OPT_LOOKAHEAD non-zero each update does the next panel's columns
 * first, then its rows, then the rest; that panel's FACT, its U12 and its
 * FP16/BF16 copies run on a second stream beside the rest of the update; the
 * factors are bitwise those of the plain schedule.
 * Workspace: 4 n nb bytes (the FP16/BF16 copies of L21 and U12), twice that
 * with look-ahead (two sets), kept per device.
 */
int hpl_mxp_factor(const double *A, int64_t n, int64_t lda, int64_t nb, int fmt, float *LU,
                   int64_t ldlu, int64_t *info, void *hip_stream);

/*
 * hpl_mxp_solve -- x from the FP32 factors, refined in FP64:
 *   x = U^{-1} L^{-1} b;  repeat  r = b - A x (FP64, explicit A);
 *   scaled = ||r||inf / (eps (||A||inf ||x||inf + ||b||inf) n), eps = 2^-53;
 *   stop if scaled < 16 or max_iter corrections were applied;
 *   d = U^{-1} L^{-1} r;  x += d.
 *   1 A device FP64 n x n at lda (the matrix that was factored); 2 lda
 *   3 LU device FP32 factors from hpl_mxp_factor; 4 ldlu
 *   5 n >= 0;  6 b device double[n];  7 x device double[n] (written)
 *   8 max_iter >= 0 corrections at most
 *   9 out host double[5] = {corrections applied, final scaled residual,
 *     ||r||inf, ||A||inf, ||x||inf}
 *  10 hip_stream
 * The run passes when out[1] < 16.
 */
int hpl_mxp_solve(const double *A, int64_t lda, const float *LU, int64_t ldlu, int64_t n,
                  const double *b, double *x, int64_t max_iter, double *out, void *hip_stream);

/* Options (process-wide, read at the start of each call). */
enum hpl_option {
    HPL_OPT_LOOKAHEAD = 1,   /* 0: none.  1: panel j+1 is factored while the RS/TRSM of
                                panel j finish; the trailing GEMM starts when the panel
                                is done.  2: the panel also overlaps the GEMM.  3
                                (default): 2 for n <= 32768, 1 above (the faster of the
                                two measured at each size).  All give the same bits.
                                hpl_mxp_factor: 1 and 2 both overlap the next FACT with
                                the trailing update (it has no RS to overlap). */
    HPL_OPT_PANEL_BASE = 2,  /* leaf width of the recursive panel: 8, 16, 32 or 64 (default 32) */
    HPL_OPT_PANEL_WGS = 3,   /* max workgroups of the panel leaf kernel, 1..256 (default 256) */
    HPL_OPT_TIMING = 4,      /* 1: time every kernel with HIP events (see hpl_get_stats) */
    HPL_OPT_PROGRESS = 5,    /* k > 0: print a progress line to stderr every k panels */
    HPL_OPT_SERIALIZE = 6,   /* 1: run every step on one stream (debug; bit-identical) */
    HPL_OPT_GEMM_TILE = 7,   /* GEMM kernel variant (default 0 = auto): 1..4 the 4x4x4 tiles
                                128x128, 128x64, 64x64, 128x32; 5, 6 the streamed 16x16x4
                                tiles 128x128, 128x64 (where their preconditions hold) */
    HPL_OPT_HOST_PANEL = 8,  /* T > 0: every panel is factored on the host by T threads
                                (hpl_host_panel; the paper's CPU FACT, Sec. III-A), the
                                panel copied to pinned host memory and back; with the
                                look-ahead the whole trailing update of panel j, GEMM
                                included, overlaps the host FACT of panel j+1.  0
                                (default): the GPU panel.  Pinned staging: 8 n nb bytes. */
    HPL_OPT_LASWP_WGS = 9,   /* g > 0: the row interchanges of the trailing columns run on at
                                most g workgroups (each loops over 8-column groups), leaving
                                the other CUs to the panel on the other stream (default 96);
                                0: one workgroup per 8 columns.  Results do not depend on it. */
    HPL_OPT_BATCH_CONFIG = 10 /* hpl_batched_solve's schedule.  0 (default): chosen from the
                                tuned table (hpl_batched_config).  k = 1 + (occ - 1) *
                                HPL_BATCH_VARIANTS + v forces occ in {1, 2} systems in
                                flight per CU and variant v for every size (what the tuner
                                measures).  The panel width and the solves' row
                                block change the rounding order, so schedules agree
                                to rounding, not bit for bit. */
};
/* Returns 0, or -1 (bad key) / -2 (bad value); the option is unchanged on error. */
int hpl_set_option(int key, int64_t value);
/* Current value of an option, or INT64_MIN for an unknown key. */
int64_t hpl_get_option(int key);

/*
 * hpl_host_panel -- the paper's CPU FACT (Sec. III-A): LU with partial
 * pivoting of an m x nb panel in HOST memory by T threads, the panel split
 * into tiles of nb rows dealt round-robin to the threads (thread 0 owns the
 * tile with the diagonal block), recursive right-looking with two halves per
 * level down to 16 columns.  The comparison variant of the GPU panel.
 *   1 P       host FP64 m x nb at ldp, overwritten by L (unit, below the
 *             diagonal) and U (on and above); the rows interchanged across
 *             all nb columns
 *   2 m >= 0; 3 1 <= nb <= m (m = 0: nothing to do); 4 ldp >= max(1, m)
 *   5 ipiv    host int32[nb]: 0-based panel rows, sequential interchanges
 *   6 threads 1 <= T <= 256
 *   7 info    host int64*: 0, or k+1 for the first exactly-zero pivot column
 * Runs on the calling thread plus T-1 threads of its own; no GPU call.
 */
int hpl_host_panel(double *P, int64_t m, int64_t nb, int64_t ldp, int32_t *ipiv, int threads, int64_t *info);

/*
 * hpl_panel_factor -- the same panel factorization on the GPU (the FACT of
 * hpl_factor: recursive panel, register-resident leaves), for comparison.
 *   1 A device FP64 m x nb at lda (overwritten as for hpl_host_panel)
 *   2 m >= 0; 3 1 <= nb <= min(m, 1024); 4 lda >= max(1, m)
 *   5 ipiv device int32[nb]; 6 info host int64*; 7 hip_stream
 */
int hpl_panel_factor(double *A, int64_t m, int64_t nb, int64_t lda, int32_t *ipiv, int64_t *info, void *hip_stream);

/*
 * hpl_batched_sizes -- the sizes of a seeded batch of systems (host only):
 * n_i = nmin + min(floor(u_i (nmax - nmin + 1)), nmax - nmin) with
 * u_i = value(seed, stream 3, i) + 1/2 in [0, 1), the generator of
 * hpl_generate.
 *   1 seed; 2 count >= 0; 3 nmin >= 1; 4 nmax >= nmin
 *   5 sizes  host int32[count] (written)
 */
int hpl_batched_sizes(uint64_t seed, int64_t count, int32_t nmin, int32_t nmax, int32_t *sizes);

/*
 * hpl_batched_solve -- count independent systems A_i X_i = B_i (the method of
 * Sec. II -- LU with partial pivoting, then the triangular solves -- applied
 * to each small system) and, optionally, the adjoint of the solve for a loss
 * whose gradient with respect to X_i is W_i: grad_B_i = A_i^{-T} W_i,
 * grad_A_i = -grad_B_i X_i^T.  ONE persistent launch for the whole batch,
 * systems taken largest first from a device-side queue.
 * Packed layout (all column-major with leading dimension n_i, device memory):
 * A_i at offset sum_{j<i} n_j^2 (elements); B_i, W_i, grad_B_i at
 * nrhs * sum_{j<i} n_j; ipiv_i at sum_{j<i} n_j (0-based within the system,
 * sequential interchanges, L in LAPACK form: P A = L U); grad_A_i like A_i.
 *   1 count >= 0
 *   2 sizes  host int32[count], 1 <= n_i <= 512
 *   3 nrhs   1 <= nrhs <= 16
 *   4 A      mode & 1: the systems, overwritten by their LU factors;
 *            mode == 2: the LU factors (input)
 *   5 ipiv   device int32[sum n_i]: written (mode & 1) or read (mode == 2)
 *   6 B      mode & 1: the right-hand sides, overwritten by X;
 *            mode == 2: X (input)
 *   7 W      mode & 2: device, layout of B (input)
 *   8 GB     mode & 2: device, layout of B (written: grad_B)
 *   9 GA     mode & 2: device, layout of A (written: grad_A)
 *  10 mode   1 = factor + solve, 2 = adjoint from stored factors and X,
 *            3 = both in the same launch
 *  11 info   host int64[count]: 0, or k+1 for the first exactly-zero pivot
 *            column of system i (that column is left unscaled)
 *  12 hip_stream
 * Workspace: 32 bytes per system (offsets, order, info), kept per device.
 * Every grid wave exits once the queue passes the batch size.
 */
int hpl_batched_solve(int64_t count, const int32_t *sizes, int64_t nrhs, double *A, int32_t *ipiv, double *B,
                      const double *W, double *GB, double *GA, int mode, int64_t *info, void *hip_stream);

/*
 * Schedules of hpl_batched_solve.  The factorization of a system comes in
 * HPL_BATCH_VARIANTS variants -- panel width PB and columns of U12 per LDS
 * stage UC of the trailing update: v = 0: PB 32, UC 128; 1: PB 32, UC 64;
 * 2: PB 16, UC 128; 3: PB 16, UC 64 -- chosen per size bucket (n - 1) / 32,
 * and the launch runs occ = 1 or 2 systems at a time on each CU (512-thread
 * workgroups; with 2, one system's per-column barriers hide behind the
 * other's work).  The library holds a table of measured costs, microseconds
 * per system amortized over the whole device, for every (occ, v, bucket),
 * written by the package's tuner (tune_batched.py) at nrhs = 4.
 *
 * hpl_batched_config -- the schedule the default option picks for a batch
 * (host only, no GPU call): per occ, each bucket takes its cheapest variant;
 * the occ whose predicted total (the sum of the systems' costs) is smaller
 * wins.
 *   1 count >= 0; 2 sizes host int32[count], 1 <= n_i <= 512
 *   3 occ    host int* (written)
 *   4 vtab   host int8[HPL_BATCH_BUCKETS] (written: the variant of each bucket)
 *   5 predicted_ms  host double* (written; may be NULL)
 */
#define HPL_BATCH_VARIANTS 4
#define HPL_BATCH_BUCKETS 16
int hpl_batched_config(int64_t count, const int32_t *sizes, int *occ, int8_t *vtab, double *predicted_ms);

/*
 * hpl_batched_table -- the tuned table itself: cost[((occ - 1) *
 * HPL_BATCH_VARIANTS + v) * HPL_BATCH_BUCKETS + bucket] in microseconds per
 * system (2 * 4 * 16 doubles), and whether it came from a tuning run (1) or
 * is the built-in default (0).
 */
int hpl_batched_table(double *cost, int *tuned);

/*
 * Per-kernel-class statistics of the calls made since the last
 * hpl_reset_stats, collected while HPL_OPT_TIMING is 1.  Entry k of the
 * arrays describes class k: 0 trailing GEMM, 1 panel (recursive FACT, all of
 * its kernels), 2 laswp, 3 trsm, 4 solve, 5 interchange plans, 6 the mixed-
 * precision trailing update, 7 the rest of a mixed-precision panel step
 * (FACT, U12, scaling and conversion), 8 hpl_solve_grad_a, 9
 * hpl_batched_solve.  For each
 * class: launches[k], total device milliseconds ms[k] (sum of HIP-event
 * intervals around each launch on the stream it ran on) and algorithmic
 * flops[k] and bytes[k] (the method's own operation and HBM byte counts).
 * Arrays are host arrays of length cap; returns the number of classes.
 */
int hpl_get_stats(int64_t *launches, double *ms, double *flops, double *bytes, int cap);
void hpl_reset_stats(void);

/*
 * hpl_mfma_peak -- measured FP64 matrix-core peak of the current device, the
 * reference next to the datasheet figure when a run is reported as a fraction
 * of peak.  Runs a pure v_mfma_f64_16x16x4_f64 issue loop (16 independent
 * accumulator blocks per wave, accumulators in AGPRs, two 256-thread
 * workgroups per CU) for `iters` rounds, three times after a warm-up, and
 * keeps the fastest.
 *   1 iters  rounds per wave, > 0 (2e5 takes about 0.2 s on MI355X).
 *   2 out    host double[2] = {TFLOP/s, milliseconds of the fastest launch}.
 *   3 hip_stream
 * Uses the library's reduction workspace (1 MB); returns after completion.
 */
int hpl_mfma_peak(int64_t iters, double *out, void *hip_stream);

/* Frees the per-device workspace, streams and events.  Returns 0 or HPL_ERR_HIP. */
int hpl_release(void);

/* Static text for a return code (negative codes name the argument position). */
const char *hpl_strerror(int code);

/* Text describing the last runtime failure in this process (HIP call, file, line). */
const char *hpl_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* HPLX_HPL_H */
