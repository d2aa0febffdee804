/*
 * oracle.c -- the CPU oracle for the HPL hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the GPU library
 * (paper_2304_10397_amd/csrc), and the GPU library never calls it.
 *
 * What it computes (Chalmers, Kurzak, McDougall, Bauman, "Optimizing
 * High-Performance Linpack for Exascale Accelerated Architectures"):
 *   - Sec. II: a random N x N double-precision system A x = b is solved by
 *     Gaussian elimination with partial pivoting, A = P L U, the system is
 *     reduced to U x = L^{-1} P^{-1} b and x is found by applying U^{-1}.
 *   - Sec. I (FACT, RS, UPDATE bullets) and Sec. II (phase descriptions): the
 *     blocked method is a reordering of the same eliminations; the oracle is
 *     the unblocked elimination, one column at a time, in the paper's order
 *     (find pivot, interchange rows, scale, update the trailing matrix).
 *   - The HPL acceptance test (scaled residual < 16) is not printed in the
 *     paper; its formula is the standard HPL one, written out in
 *     oracle_residual below.
 *
 * Precision: IEEE fp64 throughout (the paper's double precision), compiled
 * with -ffp-contract=off so every a*b+c is two correctly rounded operations.
 *
 * Beyond the paper (the differentiable form of the solve): the standard
 * normal input generator (Box-Muller) and the gradient of a linear solve,
 * oracle_normal / oracle_solve_grad at the end of the file.
 *
 * Parity pins (what ties this file to something other than itself) live in
 * tests/test_oracle_*.py: Leibniz and Bareiss determinants, exact dyadic
 * factorizations, integer systems with known solutions, special matrices,
 * LAPACK (scipy) as an independent opinion, and the published SplitMix64
 * output sequence for the generator.
 */
#define _POSIX_C_SOURCE 200809L /* pthread barriers under -std=c99 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <string.h>
#include <stdlib.h>
#include <pthread.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------ */
/* Input generator.                                                          */
/*                                                                           */
/* The paper only says the matrix is random (Sec. I, Sec. II).  The reading  */
/* used here: entries i.i.d. uniform on [-0.5, 0.5), drawn from SplitMix64   */
/* (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",    */
/* OOPSLA 2014) used as a counter-based generator: the value at linear       */
/* index idx of a stream is the idx-th output of a SplitMix64 sequence,      */
/* i.e. mix64(s0 + (idx + 1) * GAMMA), so any element can be produced on its */
/* own.  s0 for (seed, stream) is the first SplitMix64 output of the state   */
/* seed + stream * STREAM_STRIDE.                                            */
/* ------------------------------------------------------------------------ */
static const uint64_t GAMMA = 0x9E3779B97F4A7C15ull;         /* SplitMix64 increment */
static const uint64_t STREAM_STRIDE = 0xD1B54A32D192ED03ull; /* odd, separates streams */

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* idx-th output (idx = 0, 1, ...) of the SplitMix64 sequence with state s0. */
uint64_t oracle_splitmix64_at(uint64_t s0, uint64_t idx)
{
    return mix64(s0 + (idx + 1ull) * GAMMA);
}

uint64_t oracle_stream_key(uint64_t seed, uint64_t stream)
{
    return oracle_splitmix64_at(seed + stream * STREAM_STRIDE, 0);
}

/* 53 high bits -> [0,1) -> shift to [-0.5, 0.5); every step is exact. */
double oracle_uniform(uint64_t s0, uint64_t idx)
{
    uint64_t h = oracle_splitmix64_at(s0, idx);
    double u = (double)(h >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
    return u - 0.5;
}

/* M[i + j*ld] = value of linear index i + j*rows of stream (seed, stream). */
void oracle_gen(uint64_t seed, uint64_t stream, double *M, int64_t rows, int64_t cols, int64_t ld)
{
    uint64_t s0 = oracle_stream_key(seed, stream);
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t i = 0; i < rows; ++i)
            M[IDX(i, j, ld)] = oracle_uniform(s0, (uint64_t)i + (uint64_t)j * (uint64_t)rows);
}

/* ------------------------------------------------------------------------ */
/* LU factorization with partial pivoting, unblocked, right-looking.         */
/*                                                                           */
/* Column k: (1) the pivot is the row of largest |a_ik|, i >= k, the first   */
/* such row on ties; (2) rows k and p are interchanged across all n columns  */
/* (so L ends up with every later interchange applied: P A = L U with        */
/* P = S_{n-1} ... S_0, S_k swapping rows k and ipiv[k]); (3) the entries    */
/* below the diagonal are divided by the pivot; (4) the trailing matrix gets */
/* the rank-1 update a_ij -= l_ik * u_kj.  A zero pivot column leaves the     */
/* column untouched and records info = k + 1 for the first such k.           */
/* ipiv is 0-based.                                                          */
/* ------------------------------------------------------------------------ */
void oracle_lu(double *A, int64_t n, int64_t lda, int32_t *ipiv, int64_t *info)
{
    *info = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t p = k;
        double amax = fabs(A[IDX(k, k, lda)]);
        for (int64_t i = k + 1; i < n; ++i) {
            double v = fabs(A[IDX(i, k, lda)]);
            if (v > amax) { amax = v; p = i; }
        }
        ipiv[k] = (int32_t)p;
        if (amax == 0.0) {
            if (*info == 0) *info = k + 1;
            continue;
        }
        if (p != k) {
            for (int64_t j = 0; j < n; ++j) {
                double t = A[IDX(k, j, lda)];
                A[IDX(k, j, lda)] = A[IDX(p, j, lda)];
                A[IDX(p, j, lda)] = t;
            }
        }
        double piv = A[IDX(k, k, lda)];
        for (int64_t i = k + 1; i < n; ++i)
            A[IDX(i, k, lda)] = A[IDX(i, k, lda)] / piv;
        for (int64_t j = k + 1; j < n; ++j) {
            double ukj = A[IDX(k, j, lda)];
            for (int64_t i = k + 1; i < n; ++i)
                A[IDX(i, j, lda)] = A[IDX(i, j, lda)] - A[IDX(i, k, lda)] * ukj;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The same factorization on T host threads (used only to time the oracle on */
/* every core of a host).  The steps are those of oracle_lu, in the same     */
/* order: thread 0 finds the pivot, interchanges the rows and divides the    */
/* column; then the rank-1 update's columns j > k are split into T contiguous */
/* ranges, one per thread, with a barrier before and after.  Every element   */
/* receives exactly the operations of oracle_lu in the same order, so the    */
/* result is bitwise that of oracle_lu for any T.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *A;
    int64_t n, lda;
    int32_t *ipiv;
    int64_t *info;
    int threads;              /* threads taking part (those that could be started) */
    int skip;                 /* step k has an all-zero pivot column */
    int go;                   /* start gate, set once the thread count is known */
    pthread_mutex_t mu;
    pthread_cond_t cv;
    pthread_barrier_t bar;
} par_lu_t;

typedef struct {
    par_lu_t *p;
    int tid;
} par_arg_t;

/* Thread 0's part of step k: pivot search, row interchange, division. */
static void par_pivot_step(par_lu_t *p, int64_t k)
{
    double *A = p->A;
    const int64_t n = p->n, lda = p->lda;
    int64_t piv_row = k;
    double amax = fabs(A[IDX(k, k, lda)]);
    for (int64_t i = k + 1; i < n; ++i) {
        double v = fabs(A[IDX(i, k, lda)]);
        if (v > amax) { amax = v; piv_row = i; }
    }
    p->ipiv[k] = (int32_t)piv_row;
    p->skip = amax == 0.0;
    if (p->skip) {
        if (*p->info == 0) *p->info = k + 1;
        return;
    }
    if (piv_row != k) {
        for (int64_t j = 0; j < n; ++j) {
            double t = A[IDX(k, j, lda)];
            A[IDX(k, j, lda)] = A[IDX(piv_row, j, lda)];
            A[IDX(piv_row, j, lda)] = t;
        }
    }
    double piv = A[IDX(k, k, lda)];
    for (int64_t i = k + 1; i < n; ++i)
        A[IDX(i, k, lda)] = A[IDX(i, k, lda)] / piv;
}

static void *par_worker(void *arg)
{
    par_lu_t *p = ((par_arg_t *)arg)->p;
    const int tid = ((par_arg_t *)arg)->tid;
    pthread_mutex_lock(&p->mu);
    while (!p->go) pthread_cond_wait(&p->cv, &p->mu);
    pthread_mutex_unlock(&p->mu);
    double *A = p->A;
    const int64_t n = p->n, lda = p->lda, T = p->threads;
    for (int64_t k = 0; k < n; ++k) {
        if (tid == 0) par_pivot_step(p, k);
        pthread_barrier_wait(&p->bar);
        if (!p->skip) {
            /* this thread's share of the columns of the rank-1 update */
            const int64_t cols = n - k - 1;
            const int64_t j0 = k + 1 + cols * tid / T, j1 = k + 1 + cols * (tid + 1) / T;
            for (int64_t j = j0; j < j1; ++j) {
                double ukj = A[IDX(k, j, lda)];
                for (int64_t i = k + 1; i < n; ++i)
                    A[IDX(i, j, lda)] = A[IDX(i, j, lda)] - A[IDX(i, k, lda)] * ukj;
            }
        }
        pthread_barrier_wait(&p->bar);
    }
    return NULL;
}

/* threads in [1, 256]; returns the number of threads that took part (fewer  */
/* than asked if some could not be started), or -1 if nothing was computed.  */
int oracle_lu_par(double *A, int64_t n, int64_t lda, int32_t *ipiv, int64_t *info, int threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    par_lu_t p;
    p.A = A; p.n = n; p.lda = lda; p.ipiv = ipiv; p.info = info; p.skip = 0; p.go = 0;
    *info = 0;
    pthread_mutex_init(&p.mu, NULL);
    pthread_cond_init(&p.cv, NULL);
    pthread_t th[256];
    par_arg_t args[256];
    for (int t = 0; t < threads; ++t) { args[t].p = &p; args[t].tid = t; }
    int started = 1;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&th[t], NULL, par_worker, &args[t]) != 0) break;
        ++started;
    }
    p.threads = started;
    int ok = pthread_barrier_init(&p.bar, NULL, (unsigned)started) == 0;
    if (!ok) p.n = 0; /* nothing to do: every thread leaves at once */
    pthread_mutex_lock(&p.mu);
    p.go = 1;
    pthread_cond_broadcast(&p.cv);
    pthread_mutex_unlock(&p.mu);
    par_worker(&args[0]);
    for (int t = 1; t < started; ++t) pthread_join(th[t], NULL);
    if (ok) pthread_barrier_destroy(&p.bar);
    pthread_cond_destroy(&p.cv);
    pthread_mutex_destroy(&p.mu);
    return ok ? started : -1;
}

/* ------------------------------------------------------------------------ */
/* Solve with the factors (Sec. II: U x = L^{-1} P b, then x = U^{-1} ...).  */
/* trans = 0: A X = B.  Interchanges applied in order k = 0..n-1, forward    */
/*            substitution with unit L, back substitution with U.            */
/* trans = 1: A^T X = B.  Since A = P^T L U, A^T = U^T L^T P: forward with   */
/*            U^T, backward with unit L^T, interchanges in reverse order.    */
/* ------------------------------------------------------------------------ */
void oracle_solve(const double *LU, const int32_t *ipiv, double *B, int64_t n, int64_t lda,
                  int64_t nrhs, int64_t ldb, int trans)
{
    for (int64_t c = 0; c < nrhs; ++c) {
        double *b = B + (size_t)c * (size_t)ldb;
        if (trans == 0) {
            for (int64_t k = 0; k < n; ++k) {
                int64_t p = ipiv[k];
                if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
            }
            for (int64_t i = 0; i < n; ++i) {
                double s = b[i];
                for (int64_t j = 0; j < i; ++j) s = s - LU[IDX(i, j, lda)] * b[j];
                b[i] = s;
            }
            for (int64_t i = n - 1; i >= 0; --i) {
                double s = b[i];
                for (int64_t j = i + 1; j < n; ++j) s = s - LU[IDX(i, j, lda)] * b[j];
                b[i] = s / LU[IDX(i, i, lda)];
            }
        } else {
            /* U^T z = b: (U^T)_{ij} = u_ji, lower triangular with diagonal u_ii */
            for (int64_t i = 0; i < n; ++i) {
                double s = b[i];
                for (int64_t j = 0; j < i; ++j) s = s - LU[IDX(j, i, lda)] * b[j];
                b[i] = s / LU[IDX(i, i, lda)];
            }
            /* L^T w = z: (L^T)_{ij} = l_ji, unit upper triangular */
            for (int64_t i = n - 1; i >= 0; --i) {
                double s = b[i];
                for (int64_t j = i + 1; j < n; ++j) s = s - LU[IDX(j, i, lda)] * b[j];
                b[i] = s;
            }
            for (int64_t k = n - 1; k >= 0; --k) {
                int64_t p = ipiv[k];
                if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* HPL scaled residual: ||A x - b||_inf / (eps * (||A||_inf ||x||_inf +      */
/* ||b||_inf) * n), eps = 2^-53 (unit roundoff of fp64).  out[5] =           */
/* {scaled, ||r||_inf, ||A||_inf, ||x||_inf, ||b||_inf}; with several right- */
/* hand sides out[0] is the largest per-column scaled residual and out[1],   */
/* out[3], out[4] the largest per-column norms.                              */
/* The matrix is either given (A != NULL) or regenerated from (seed, 0).     */
/* ------------------------------------------------------------------------ */
static void residual_impl(const double *A, int64_t lda, int gen, uint64_t seed, int64_t n,
                          const double *X, int64_t ldx, const double *B, int64_t ldb,
                          int64_t nrhs, double *out)
{
    const double eps = 1.0 / 9007199254740992.0;
    uint64_t s0 = gen ? oracle_stream_key(seed, 0) : 0;
    double anorm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double a = gen ? oracle_uniform(s0, (uint64_t)i + (uint64_t)j * (uint64_t)n)
                           : A[IDX(i, j, lda)];
            rs = rs + fabs(a);
        }
        if (!(rs <= anorm)) anorm = rs; /* NaN propagates */
    }
    double worst = 0.0, rmax = 0.0, xmax = 0.0, bmax = 0.0;
    for (int64_t c = 0; c < nrhs; ++c) {
        const double *x = X + (size_t)c * (size_t)ldx;
        const double *b = B + (size_t)c * (size_t)ldb;
        double rn = 0.0, xn = 0.0, bn = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double a = gen ? oracle_uniform(s0, (uint64_t)i + (uint64_t)j * (uint64_t)n)
                               : A[IDX(i, j, lda)];
                s = s + a * x[j];
            }
            double r = fabs(s - b[i]);
            if (!(r <= rn)) rn = r;
            if (!(fabs(x[i]) <= xn)) xn = fabs(x[i]);
            if (!(fabs(b[i]) <= bn)) bn = fabs(b[i]);
        }
        double scaled = rn / (eps * (anorm * xn + bn) * (double)n);
        if (!(scaled <= worst)) worst = scaled;
        if (!(rn <= rmax)) rmax = rn;
        if (!(xn <= xmax)) xmax = xn;
        if (!(bn <= bmax)) bmax = bn;
    }
    out[0] = worst; out[1] = rmax; out[2] = anorm; out[3] = xmax; out[4] = bmax;
}

void oracle_residual(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                     const double *B, int64_t ldb, int64_t nrhs, double *out)
{
    residual_impl(A, lda, 0, 0, n, X, ldx, B, ldb, nrhs, out);
}

void oracle_residual_gen(uint64_t seed, int64_t n, const double *X, int64_t ldx,
                         const double *B, int64_t ldb, int64_t nrhs, double *out)
{
    residual_impl(NULL, 0, 1, seed, n, X, ldx, B, ldb, nrhs, out);
}

/* ------------------------------------------------------------------------ */
/* Determinant from the factors: det A = (-1)^s * prod u_kk, s = number of   */
/* k with ipiv[k] != k (each is one interchange).  Returned as sign, and the */
/* sum of log2 |u_kk| so that large n does not overflow; *exact holds the    */
/* plain product when it is finite.                                          */
/* ------------------------------------------------------------------------ */
void oracle_det(const double *LU, const int32_t *ipiv, int64_t n, int64_t lda,
                double *sign, double *log2abs, double *exact)
{
    double s = 1.0, l2 = 0.0, prod = 1.0;
    for (int64_t k = 0; k < n; ++k) {
        double u = LU[IDX(k, k, lda)];
        if (ipiv[k] != k) s = -s;      /* one interchange */
        if (u < 0) s = -s;
        l2 += log2(fabs(u));
        prod = prod * u;
    }
    *sign = s;
    *log2abs = l2;
    *exact = s * fabs(prod);
}

/* ------------------------------------------------------------------------ */
/* Standard normal input (the weights W of the differentiable solve's loss). */
/* Box-Muller transform (Box and Muller, 1958) of two uniforms of the stream */
/* at the SplitMix64 outputs 2 idx and 2 idx + 1:                            */
/*   u1 = (h(2 idx) >> 11) 2^-53,  u2 = (h(2 idx + 1) >> 11) 2^-53 in [0,1), */
/*   z  = sqrt(-2 ln(1 - u1)) cos(2 pi u2)                                   */
/* (1 - u1 lies in (0, 1], so the logarithm is finite).  The value depends   */
/* on the C library's log and cos; another implementation of the same        */
/* formula agrees to a few units in the last place, not bit for bit.         */
/* ------------------------------------------------------------------------ */
double oracle_normal(uint64_t s0, uint64_t idx)
{
    const double u1 = (double)(oracle_splitmix64_at(s0, 2 * idx) >> 11) * 0x1.0p-53;
    const double u2 = (double)(oracle_splitmix64_at(s0, 2 * idx + 1) >> 11) * 0x1.0p-53;
    const double two_pi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(1.0 - u1)) * cos(two_pi * u2);
}

/* M[i + j*ld] = normal value of linear index i + j*rows of stream (seed, stream). */
void oracle_gen_normal(uint64_t seed, uint64_t stream, double *M, int64_t rows, int64_t cols, int64_t ld)
{
    const uint64_t s0 = oracle_stream_key(seed, stream);
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t i = 0; i < rows; ++i) M[IDX(i, j, ld)] = oracle_normal(s0, (uint64_t)(i + j * rows));
}

/* ------------------------------------------------------------------------ */
/* Gradient of a linear solve.  For X = A^{-1} B and a loss L(X) whose       */
/* gradient with respect to X is W (for L = sum_ij W_ij X_ij that is W       */
/* itself), differentiating A X = B gives A dX = dB - dA X, so               */
/*   dL = <W, dX> = <A^{-T} W, dB> - <(A^{-T} W) X^T, dA>,                   */
/* i.e. grad_B = A^{-T} W and grad_A = -grad_B X^T.  The oracle takes the    */
/* steps literally: factor a copy of A (oracle_lu), X by the forward solve,  */
/* grad_B by the transposed solve with the same factors, grad_A as the       */
/* explicit outer product summed over the right-hand sides in order.         */
/* Outputs X (n x nrhs at ldx), GB (n x nrhs at ldgb), GA (n x n at ldga).   */
/* Returns info of the factorization (0, or k+1 for a zero pivot).           */
/* oracle_solve_grad_par is the same with the factorization on `threads`     */
/* host threads (oracle_lu_par: bitwise the factors of oracle_lu), for the   */
/* large systems whose reference would otherwise take minutes.               */
/* ------------------------------------------------------------------------ */
static int64_t solve_grad_impl(const double *A, int64_t n, int64_t lda, const double *B, int64_t ldb,
                               int64_t nrhs, const double *W, int64_t ldw, double *X, int64_t ldx, double *GB,
                               int64_t ldgb, double *GA, int64_t ldga, int threads)
{
    if (n <= 0) return 0;
    double *LU = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    int32_t *ipiv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t info = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) LU[IDX(i, j, n)] = A[IDX(i, j, lda)];
    if (threads > 1) {
        if (oracle_lu_par(LU, n, n, ipiv, &info, threads) < 1) oracle_lu(LU, n, n, ipiv, &info);
    } else {
        oracle_lu(LU, n, n, ipiv, &info);
    }
    for (int64_t r = 0; r < nrhs; ++r)
        for (int64_t i = 0; i < n; ++i) {
            X[IDX(i, r, ldx)] = B[IDX(i, r, ldb)];
            GB[IDX(i, r, ldgb)] = W[IDX(i, r, ldw)];
        }
    oracle_solve(LU, ipiv, X, n, n, nrhs, ldx, 0);
    oracle_solve(LU, ipiv, GB, n, n, nrhs, ldgb, 1);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t r = 0; r < nrhs; ++r) s = s + GB[IDX(i, r, ldgb)] * X[IDX(j, r, ldx)];
            GA[IDX(i, j, ldga)] = -s;
        }
    free(LU);
    free(ipiv);
    return info;
}

int64_t oracle_solve_grad(const double *A, int64_t n, int64_t lda, const double *B, int64_t ldb, int64_t nrhs,
                          const double *W, int64_t ldw, double *X, int64_t ldx, double *GB, int64_t ldgb,
                          double *GA, int64_t ldga)
{
    return solve_grad_impl(A, n, lda, B, ldb, nrhs, W, ldw, X, ldx, GB, ldgb, GA, ldga, 1);
}

int64_t oracle_solve_grad_par(const double *A, int64_t n, int64_t lda, const double *B, int64_t ldb,
                              int64_t nrhs, const double *W, int64_t ldw, double *X, int64_t ldx, double *GB,
                              int64_t ldgb, double *GA, int64_t ldga, int threads)
{
    return solve_grad_impl(A, n, lda, B, ldb, nrhs, W, ldw, X, ldx, GB, ldgb, GA, ldga, threads);
}

/* ------------------------------------------------------------------------ */
/* Mixed precision (HPL-MxP, the paper's Sec. I mention of the mixed-        */
/* precision benchmark).  The input is diagonally dominant so that LU needs  */
/* no pivoting: a_ij uniform on [-0.5, 0.5) as above, then                   */
/* a_ii := sum_j |a_ij| over the row as generated (diagonal included).       */
/* ------------------------------------------------------------------------ */
void oracle_mxp_gen(uint64_t seed, double *A, int64_t n, int64_t lda)
{
    oracle_gen(seed, 0, A, n, n, lda);
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s = s + fabs(A[IDX(i, j, lda)]);
        A[IDX(i, i, lda)] = s;
    }
}

/* IEEE binary16 (1 sign, 5 exponent, 10 fraction bits) rounding of a float, */
/* round to nearest, ties to even, with gradual underflow and overflow to    */
/* infinity: written from the format's definition, value returned as float.  */
float oracle_round_fp16(float x)
{
    if (!(x == x) || x == 0.0f) return x;
    const double ax = fabs((double)x);
    if (ax >= 65520.0) return x > 0 ? INFINITY : -INFINITY;  /* 65504 + half an ulp rounds up */
    int e;
    frexp(ax, &e);                        /* ax = m 2^e, m in [0.5, 1) */
    int q = e - 11;                       /* ulp exponent for 11 significant bits */
    if (q < -24) q = -24;                 /* subnormal spacing 2^-24 */
    const double scaled = ldexp(ax, -q);  /* exact: a power-of-two scaling */
    double r = floor(scaled);
    const double frac = scaled - r;
    if (frac > 0.5 || (frac == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
    const double v = ldexp(r, q);
    return (float)(x < 0 ? -v : v);
}

/* bfloat16 (the top 16 bits of binary32): round to nearest, ties to even on */
/* the 16 discarded bits.                                                    */
float oracle_round_bf16(float x)
{
    if (!(x == x)) return x;
    uint32_t u;
    memcpy(&u, &x, 4);
    const uint32_t lower = u & 0xFFFFu;
    uint32_t upper = u >> 16;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) upper += 1u;
    u = upper << 16;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static float round_fmt(float x, int fmt)
{
    return fmt == 0 ? oracle_round_fp16(x) : (fmt == 1 ? oracle_round_bf16(x) : x);
}

/* Exponent s of the per-panel scaling: L21 is multiplied by 2^s and U12 by  */
/* 2^-s (exact), s = round((log2 max|U12| - log2 max|L21|) / 2), so both      */
/* operands sit around the geometric mean of their magnitudes.                */
static int mxp_scale_exponent(float lmax, float umax)
{
    if (!(lmax > 0.0f) || !(umax > 0.0f)) return 0;
    int el, eu;
    frexpf(lmax, &el);
    frexpf(umax, &eu);
    const int d = eu - el;
    return d >= 0 ? (d + 1) / 2 : -((-d + 1) / 2);
}

/* LU without pivoting in the method's mixed precision, blocked right-looking */
/* with panel width nb, the steps in order for each panel [c0, c1):           */
/*  1. FACT: column by column in FP32 (divide by the diagonal, rank-1 update  */
/*     of the panel's remaining columns);                                     */
/*  2. U12 = L11^{-1} A12 by forward substitution in FP32;                    */
/*  3. UPDATE: A22 += (-(2^s L21) rounded to the format) x ((2^-s U12)        */
/*     rounded to the format), products of the rounded operands summed in     */
/*     FP32 over k in order (fmt 0 = FP16, 1 = BF16, 2 = no rounding).        */
/* A (double, n x n at lda) is the input; LU (float, n x n at ldlu) receives  */
/* the unit-lower L below the diagonal and U on and above it.  Returns info   */
/* (k+1 for the first zero diagonal, whose column is then left unscaled).     */
int64_t oracle_lu_mxp(const double *A, int64_t n, int64_t lda, int64_t nb, int fmt, float *LU, int64_t ldlu)
{
    int64_t info = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) LU[IDX(i, j, ldlu)] = (float)A[IDX(i, j, lda)];
    float *lo = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1) * (size_t)(nb > 0 ? nb : 1));
    float *up = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1) * (size_t)(nb > 0 ? nb : 1));
    for (int64_t c0 = 0; c0 < n; c0 += nb) {
        const int64_t c1 = (c0 + nb < n) ? c0 + nb : n, w = c1 - c0;
        /* 1. panel */
        for (int64_t k = c0; k < c1; ++k) {
            const float piv = LU[IDX(k, k, ldlu)];
            if (piv == 0.0f) {
                if (!info) info = k + 1;
                continue;
            }
            for (int64_t i = k + 1; i < n; ++i) LU[IDX(i, k, ldlu)] = LU[IDX(i, k, ldlu)] / piv;
            for (int64_t j = k + 1; j < c1; ++j) {
                const float ukj = LU[IDX(k, j, ldlu)];
                for (int64_t i = k + 1; i < n; ++i) LU[IDX(i, j, ldlu)] = LU[IDX(i, j, ldlu)] - LU[IDX(i, k, ldlu)] * ukj;
            }
        }
        if (c1 >= n) break;
        /* 2. U12 */
        for (int64_t j = c1; j < n; ++j)
            for (int64_t i = c0; i < c1; ++i) {
                float s = LU[IDX(i, j, ldlu)];
                for (int64_t k = c0; k < i; ++k) s = s - LU[IDX(i, k, ldlu)] * LU[IDX(k, j, ldlu)];
                LU[IDX(i, j, ldlu)] = s;
            }
        /* 3. scaled, rounded operands and the FP32 update */
        float lmax = 0.0f, umax = 0.0f;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t i = c1; i < n; ++i) {
                const float v = fabsf(LU[IDX(i, c0 + k, ldlu)]);
                if (v > lmax) lmax = v;
            }
        for (int64_t j = c1; j < n; ++j)
            for (int64_t k = 0; k < w; ++k) {
                const float v = fabsf(LU[IDX(c0 + k, j, ldlu)]);
                if (v > umax) umax = v;
            }
        const int s = mxp_scale_exponent(lmax, umax);
        const int64_t m = n - c1;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t i = 0; i < m; ++i) lo[IDX(i, k, m)] = round_fmt(-ldexpf(LU[IDX(c1 + i, c0 + k, ldlu)], s), fmt);
        for (int64_t j = 0; j < m; ++j)
            for (int64_t k = 0; k < w; ++k) up[IDX(k, j, w)] = round_fmt(ldexpf(LU[IDX(c0 + k, c1 + j, ldlu)], -s), fmt);
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) {
                float acc = LU[IDX(c1 + i, c1 + j, ldlu)];
                for (int64_t k = 0; k < w; ++k) acc = acc + lo[IDX(i, k, m)] * up[IDX(k, j, w)];
                LU[IDX(c1 + i, c1 + j, ldlu)] = acc;
            }
    }
    free(lo);
    free(up);
    return info;
}
