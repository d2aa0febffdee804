// mxp.hip -- mixed-precision LU (HPL-MxP, mentioned in the paper's Sec. I)
// with FP64 iterative refinement.
//
// The input is diagonally dominant (a_ii = sum_j |a_ij| of the generated row),
// so the factorization needs no pivoting.  The working matrix is FP32 and the
// factorization is right-looking with NB-column panels:
//   1. FACT in FP32: recursive halves; leaves of <= 32 columns factor their
//      diagonal block in LDS and solve the rows below against it;
//   2. U12 = L11^{-1} A12 in FP32 (recursive: 64-row leaf solves in LDS,
//      FP32 GEMMs between them);
//   3. UPDATE on the matrix cores: L21 and U12 are scaled by 2^s and 2^-s (a
//      power of two chosen on the device from their maxima, so the scaling is
//      exact and keeps FP16 multipliers out of the subnormal range), rounded
//      to FP16 or BF16, and A22 += (-L21) U12 runs on
//      v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.
// The solution is then refined in FP64: r = b - A x with the FP64 matrix, a
// correction from the FP32 factors, x += d, until the FP64 scaled residual is
// below 16.
#include "common.hpp"

namespace hplx {

namespace {

// ---------------------------------------------------------------------------
// input: a_ii = sum_j |a_ij| over the row as generated (j in order, no FMA)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mxp_diag_kernel(double *__restrict__ A, int64_t n, int64_t lda)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s = s + fabs(A[off(i, j, lda)]);
    A[off(i, i, lda)] = s;
}

// FP64 -> FP32 copy: each thread converts rows 2i, 2i+1 of kCvCols columns
// (16-byte loads and 8-byte stores when both leading dimensions are even)
constexpr int kCvCols = 8;

template <bool VEC>
__global__ __launch_bounds__(256) void cvt_f64_f32_kernel(const double *__restrict__ A, int64_t lda,
                                                          float *__restrict__ B, int64_t ldb, int64_t rows,
                                                          int64_t cols)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float fl2 __attribute__((ext_vector_type(2)));
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 2;
    if (i >= rows) return;
    const bool pair = i + 1 < rows;
    for (int64_t j0 = (int64_t)blockIdx.y * kCvCols; j0 < cols; j0 += (int64_t)gridDim.y * kCvCols) {
#pragma unroll
        for (int c = 0; c < kCvCols; ++c) {
            const int64_t j = j0 + c;
            if (j >= cols) break;
            if (VEC && pair) {
                const d2 v = *(const d2 *)(A + off(i, j, lda));
                *(fl2 *)(B + off(i, j, ldb)) = (fl2){(float)v[0], (float)v[1]};
            } else {
                B[off(i, j, ldb)] = (float)A[off(i, j, lda)];
                if (pair) B[off(i + 1, j, ldb)] = (float)A[off(i + 1, j, lda)];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 panel leaf (w <= LW = 32 or 64 columns, rows [c, n)), no pivoting.
// Every row takes the same right-looking steps: at step k a row i > k divides
// its entry k by u_kk and subtracts that multiple of the pivot row from its
// entries q > k (a zero u_kk leaves the column as is; info reports it).  Each
// thread holds one row in registers: in every workgroup, threads 0..LW-1 hold
// the rows of the w x w diagonal block (recomputed by each workgroup) and
// threads LW..255 the rows below it, 256 - LW per workgroup.  At step k thread k publishes its row (the
// final row k of U) to a double-buffered LDS row, so one barrier per step
// suffices.  Every workgroup reads the diagonal block as input, so it is
// written back only by the last workgroup to finish (counted on *done, which
// wraps to zero at the end of each launch).  With mx, the largest |l| of the
// rows from l21_row0 on (the panel's L21) is folded into *mx (the bit pattern
// of a non-negative float), one atomicMax per workgroup.
// ---------------------------------------------------------------------------
// largest v over the workgroup into *mx (non-negative floats order as their bit
// patterns); red holds one float per wave
__device__ __forceinline__ void block_max_to(float v, unsigned *mx, float *red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    const int nw = (int)(blockDim.x >> 6);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = red[0];
        for (int q = 1; q < nw; ++q) m = fmaxf(m, red[q]);
        atomicMax(mx, __float_as_uint(m));
    }
}

template <int LW>
__global__ __launch_bounds__(256) void panel32_leaf_kernel(float *__restrict__ A, int64_t lda, int64_t c,
                                                           int64_t n, int w, unsigned long long *__restrict__ info,
                                                           unsigned *__restrict__ done, unsigned *__restrict__ mx,
                                                           int64_t l21_row0)
{
    __shared__ float red[4];
    constexpr int kLw = LW, kLeafRows = 256 - LW;
    __shared__ float P[2][kLw];
    __shared__ int last;
    const int t = threadIdx.x;
    const bool diag = t < kLw;
    // row of this thread: the diagonal block's row t, or a row below the block
    const int64_t i = diag ? c + t : c + w + (int64_t)blockIdx.x * kLeafRows + (t - kLw);
    const bool live = diag ? t < w : i < n;
    const int64_t ir = live ? i : c;  // loads from a valid row when idle
    float x[kLw];
#pragma unroll
    for (int j = 0; j < kLw; ++j) x[j] = A[off(ir, c + (j < w ? j : 0), lda)];
    unsigned first_zero = 0;
#pragma unroll
    for (int k = 0; k < kLw; ++k) {
        if (k < w) {  // uniform; the loop stays unrolled so x[] stays in registers
            if (t == k) {
#pragma unroll
                for (int q = k; q < kLw; ++q) P[k & 1][q] = x[q];
            }
            __syncthreads();
            const float ukk = P[k & 1][k];
            if (t == 0 && ukk == 0.0f && first_zero == 0) first_zero = (unsigned)k + 1;
            // rows below k: the diagonal block's rows t > k and every row below it
            // slots past w hold copies of column 0 and published values that
            // are never stored: they are updated without a test per slot
            if ((!diag || t > k) && ukk != 0.0f) {
                x[k] = x[k] / ukk;
#pragma unroll
                for (int q = k + 1; q < kLw; ++q) x[q] = x[q] - x[k] * P[k & 1][q];
            }
        }
    }
    // every thread's loads were consumed by the steps above
    __syncthreads();
    if (t == 0) {
        __threadfence();
        last = atomicInc(done, gridDim.x - 1) == gridDim.x - 1;
        if (last && first_zero != 0) atomicMin(info, (unsigned long long)(c + first_zero));
    }
    __syncthreads();
    if (live && (!diag || last)) {
#pragma unroll
        for (int j = 0; j < kLw; ++j)
            if (j < w) A[off(i, c + j, lda)] = x[j];
    }
    if (mx) {  // uniform
        float am = 0.0f;
        if (live && !diag && i >= l21_row0) {
#pragma unroll
            for (int j = 0; j < kLw; ++j)
                if (j < w) am = fmaxf(am, fabsf(x[j]));
        }
        block_max_to(am, mx, red);
    }
}

// ---------------------------------------------------------------------------
// FP32 triangular-solve leaf: B (nbk x ncols, nbk <= TL = 32 or 64) <- L^{-1} B
// with L unit lower; with mx, the largest |x| of the solution is folded into
// *mx.  A workgroup of 128 threads takes 128 columns: the TL x 128 block
// moves between B and LDS with coalesced accesses (16-byte vectors when every
// column starts 16-byte aligned, else 32 lanes per column), then each thread
// solves its column in registers, right-looking: at step k every row i > k
// subtracts l_ik x_k, so each element takes its subtractions in k order.  L is
// staged transposed so that step k reads one contiguous column of L.
// ---------------------------------------------------------------------------
constexpr int kTlCols = 128, kTlPad = 4;

template <int TL, bool VEC>
__global__ __launch_bounds__(kTlCols) void trsm32_leaf_kernel(const float *__restrict__ L, int64_t ldl,
                                                              float *__restrict__ B, int64_t ldb, int nbk,
                                                              int64_t ncols, unsigned *__restrict__ mx)
{
    __shared__ float red[kTlCols / 64];
    constexpr int kTl = TL;
    typedef float f4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) float Lt[kTl][kTl + kTlPad];            // Lt[k][i] = l_ik
    __shared__ __attribute__((aligned(16))) float Xs[kTlCols][kTl + kTlPad];        // Xs[c][i] = b_i of column c
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * kTlCols;
    constexpr int kLq = kTl * kTl / kTlCols;
    float sv[kLq];  // all loads in flight before the first LDS store
#pragma unroll
    for (int q = 0; q < kLq; ++q) {
        const int e = t + kTlCols * q, r = e % kTl, cc = e / kTl;
        sv[q] = load_or(r < nbk && cc < nbk, L + off(r, cc, ldl), L, 0.0f);
    }
    constexpr int kUc = kTl / 4;  // 16-byte units per column
    if (VEC) {
        // unit u: column u / kUc, rows 4 (u % kUc) .. + 3 (nbk == TL)
        f4 vv[kTl / 4];
#pragma unroll
        for (int q = 0; q < kTl / 4; ++q) {
            const int u = t + kTlCols * q, c = u / kUc, r4 = (u % kUc) * 4;
            const int64_t jj = j0 + c;
            const f4 v = *(const f4 *)(B + (size_t)(jj < ncols ? jj : ncols - 1) * (size_t)ldb + r4);
            vv[q] = jj < ncols ? v : (f4){0.0f, 0.0f, 0.0f, 0.0f};
        }
#pragma unroll
        for (int q = 0; q < kTl / 4; ++q) {
            const int u = t + kTlCols * q;
            *(f4 *)&Xs[u / kUc][(u % kUc) * 4] = vv[q];
        }
    } else {
        float xv[kTl];
#pragma unroll
        for (int q = 0; q < kTl; ++q) {
            const int e = t + kTlCols * q, c = e / kTl, r = e % kTl;
            const int64_t jj = j0 + c;
            const bool ok = r < nbk && jj < ncols;
            xv[q] = load_or(ok, B + (size_t)(ok ? jj : 0) * (size_t)ldb + (ok ? r : 0), B, 0.0f);
        }
#pragma unroll
        for (int q = 0; q < kTl; ++q) {
            const int e = t + kTlCols * q;
            Xs[e / kTl][e % kTl] = xv[q];
        }
    }
#pragma unroll
    for (int q = 0; q < kLq; ++q) {
        const int e = t + kTlCols * q;
        Lt[e / kTl][e % kTl] = sv[q];
    }
    __syncthreads();
    float x[kTl];
#pragma unroll
    for (int i4 = 0; i4 < kTl; i4 += 4) {
        const f4 v = *(const f4 *)&Xs[t][i4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[i4 + r] = v[r];
    }
#pragma unroll
    for (int k = 0; k < kTl - 1; ++k) {
        const float xk = x[k];
#pragma unroll
        for (int i = k + 1; i < kTl; ++i) x[i] = x[i] - Lt[k][i] * xk;
    }
#pragma unroll
    for (int i4 = 0; i4 < kTl; i4 += 4) *(f4 *)&Xs[t][i4] = (f4){x[i4], x[i4 + 1], x[i4 + 2], x[i4 + 3]};
    if (mx) {  // uniform
        float am = 0.0f;
        if (j0 + t < ncols) {
#pragma unroll
            for (int i = 0; i < kTl; ++i)
                if (i < nbk) am = fmaxf(am, fabsf(x[i]));
        }
        block_max_to(am, mx, red);  // includes the barrier before the stores below
    }
    __syncthreads();
    if (VEC) {
#pragma unroll
        for (int q = 0; q < kTl / 4; ++q) {
            const int u = t + kTlCols * q, c = u / kUc, r4 = (u % kUc) * 4;
            const int64_t jj = j0 + c;
            if (jj < ncols) *(f4 *)(B + (size_t)jj * (size_t)ldb + r4) = *(const f4 *)&Xs[c][r4];
        }
    } else {
#pragma unroll
        for (int q = 0; q < kTl; ++q) {
            const int e = t + kTlCols * q, c = e / kTl, r = e % kTl;
            const int64_t jj = j0 + c;
            if (r < nbk && jj < ncols) B[(size_t)jj * (size_t)ldb + r] = Xs[c][r];
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 GEMM C(m x n) -= A(m x k) B(k x n), column-major, for the panel and
// triangular-solve recursions: 64 x 64 tiles, 256 threads of 4 x 4 outputs,
// k staged 16 at a time through LDS; the next k tile is loaded into registers
// while the current one is multiplied.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sgemm32_kernel(int64_t m, int64_t n, int64_t k, const float *__restrict__ A,
                                                      int64_t lda, const float *__restrict__ B, int64_t ldb,
                                                      float *__restrict__ C, int64_t ldc)
{
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int t = threadIdx.x, tx = t % 16, ty = t / 16;
    const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
    float acc[4][4] = {};
    float ra[4], rb[4];
    // element u of this thread: A row (t % 64), k (t / 64 + 4u); B k (t % 16), column (t / 16 + 16u)
    auto load = [&](int64_t k0) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = t % 64, q = t / 64 + 4 * u;
            ra[u] = (m0 + r < m && k0 + q < k) ? A[off(m0 + r, k0 + q, lda)] : 0.0f;
            const int q2 = t % 16, c2 = t / 16 + 16 * u;
            rb[u] = (k0 + q2 < k && n0 + c2 < n) ? B[off(k0 + q2, n0 + c2, ldb)] : 0.0f;
        }
    };
    load(0);
    for (int64_t k0 = 0; k0 < k; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[t / 64 + 4 * u][t % 64] = ra[u];
            Bs[t % 16][t / 16 + 16 * u] = rb[u];
        }
        __syncthreads();
        if (k0 + 16 < k) load(k0 + 16);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[q][tx + 16 * u];
                b[u] = Bs[q][ty + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
        }
        __syncthreads();
    }
    // every C value is loaded (from clamped indexes) before the first store
    float cv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = m0 + tx + 16 * u, j = n0 + ty + 16 * v;
            cv[u][v] = C[off(i < m ? i : m - 1, j < n ? j : n - 1, ldc)];
        }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = m0 + tx + 16 * u, j = n0 + ty + 16 * v;
            if (i < m && j < n) C[off(i, j, ldc)] = cv[u][v] - acc[u][v];
        }
}

template <int FMT> struct Half;
template <> struct Half<0> { typedef _Float16 T; };
template <> struct Half<1> { typedef __bf16 T; };

// Layout of the low-precision operands.  Both are stored as rows of k (a row
// of A16 is a row of -L21, a row of B16 a column of U12) in 1 KB blocks of 16
// rows x 32 k, row r of a block at 64 r bytes; the blocks are ordered by k
// slab, then by 16-row group:
//     element (i, k) at  (k / 32) * ss + (i / 16) * 512 + (i % 16) * 32 + k % 32
// with ss the slab stride in elements (a multiple of 512).  One 32-k stage of
// a tile is then a run of whole 1 KB blocks, each moved by one 64-lane
// 16-byte load, and the operands of two panels sit side by side in k (panel 2
// in the slabs after panel 1's), so that one update can take both.
__device__ __forceinline__ size_t blk_index(int64_t i, int64_t k, int64_t ss)
{
    return (size_t)(k >> 5) * (size_t)ss + (size_t)(i >> 4) * 512 + (size_t)((i & 15) * 32 + (k & 31));
}

// The scaling exponent of a panel from the maxima of |L21| and |U12| (bit
// patterns of non-negative floats in mx[0], mx[1]): s = round((e_U - e_L) / 2)
// of their binary exponents, ties away from zero; 0 if either is zero.
__device__ __forceinline__ int mxp_scale_exp(const unsigned *mx)
{
    const float lmax = __uint_as_float(mx[0]), umax = __uint_as_float(mx[1]);
    if (!(lmax > 0.0f && umax > 0.0f)) return 0;
    int el, eu;
    frexpf(lmax, &el);
    frexpf(umax, &eu);
    const int d = eu - el;
    return d >= 0 ? (d + 1) / 2 : -((-d + 1) / 2);
}

// One launch for both copies of a panel, the scaling exponent computed from
// the maxima by every workgroup:
//  * blocks [0, gl gk): L21 (m x w at ldl) -> A16 (blocked, slab stride sa),
//    -(2^s l) rounded; a 64 x 64 tile goes through LDS: read down the
//    columns, written along rows;
//  * the rest: U12 (w x n at ldu) -> B16 (blocked, slab stride sb; row j of
//    B16 is column j of U12), 2^-s u rounded; each 512 consecutive threads
//    fill one block: reads of 32 consecutive k of a column, the block written
//    whole.
// Block 0 also clears the other pair of maxima (reset), which the next panel's
// maxima accumulate into.
template <int FMT>
__global__ __launch_bounds__(256) void cvt_lu_kernel(const float *__restrict__ L, int64_t ldl, int64_t m, int w,
                                                     const float *__restrict__ U, int64_t ldu, int64_t n,
                                                     const unsigned *__restrict__ mx, unsigned *__restrict__ reset,
                                                     typename Half<FMT>::T *__restrict__ A16, int64_t sa,
                                                     typename Half<FMT>::T *__restrict__ B16, int64_t sb, int64_t gl,
                                                     int64_t gk)
{
    typedef typename Half<FMT>::T H;
    __shared__ float tile[64][65];
    const int s = mxp_scale_exp(mx);
    if (blockIdx.x == 0 && threadIdx.x < 2) reset[threadIdx.x] = 0u;
    const int64_t b = blockIdx.x;
    if (b < gl * gk) {
        const int64_t i0 = (b % gl) * 64;
        const int k0 = (int)(b / gl) * 64;
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e % 64, q = e / 64;
            tile[r][q] = (i0 + r < m && k0 + q < w) ? L[off(i0 + r, k0 + q, ldl)] : 0.0f;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int q = e % 64, r = e / 64;
            if (i0 + r < m && k0 + q < w) A16[blk_index(i0 + r, k0 + q, sa)] = (H)(-ldexpf(tile[r][q], s));
        }
        return;
    }
    const int64_t e = (b - gl * gk) * 256 + threadIdx.x;
    const int64_t nbj = (n + 15) / 16;  // 16-column groups
    const int64_t blk = e >> 9, kb = blk / nbj, jb = blk - kb * nbj;
    const int within = (int)(e & 511);
    const int64_t j = jb * 16 + (within >> 5), k = kb * 32 + (within & 31);
    if (kb * 32 >= w || j >= n || k >= w) return;
    B16[(size_t)kb * (size_t)sb + (size_t)jb * 512 + within] = (H)ldexpf(U[off(k, j, ldu)], -s);
}

// ---------------------------------------------------------------------------
// Trailing update on the matrix cores: C (FP32, column-major) += A16 B16^T,
// A16 (m rows) and B16 (n rows) blocked with slab strides sa and sb.
// Tile 128 x 128, 4 waves of 64 x 64 (4 x 4 blocks of 16 x 16); K staged 64 at
// a time through double-buffered LDS (rows padded by 8 halves).  B's fragment
// is the MFMA's first operand, so a block comes out transposed: register r of
// lane l holds C(16R + l%16, 16G + 4(l/16) + r) -- 16 consecutive rows of 4
// columns.  The accumulators start at zero and C is added once at the end, as
// in the 256 x 128 kernel: the two take the same MFMAs in the same k order, so
// an element gets the same bits from either.  Requires K % 64 == 0.
// ---------------------------------------------------------------------------
constexpr int kHBM = 128, kHBN = 128, kHBK = 64, kHPad = 8;
constexpr int64_t kHGroupM = 8;  // tile-rows per group of the XCD-aware order

template <int FMT>
__global__ __launch_bounds__(256, 2) void hgemm_update_kernel(int64_t m, int64_t n, int64_t K,
                                                              const typename Half<FMT>::T *__restrict__ A16,
                                                              int64_t sa,
                                                              const typename Half<FMT>::T *__restrict__ B16,
                                                              int64_t sb, float *__restrict__ C, int64_t ldc,
                                                              int64_t tiles_m)
{
    typedef typename Half<FMT>::T H;
    typedef H h8 __attribute__((ext_vector_type(8)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    asm volatile("" ::: "a0");
    __shared__ __attribute__((aligned(16))) H As[2][kHBM][kHBK + kHPad];
    __shared__ __attribute__((aligned(16))) H Bs[2][kHBN][kHBK + kHPad];
    // XCD-aware tile order: the workgroups resident on one XCD at a time cover
    // a compact block of tiles, which share A row-panels and B column-panels
    // in that XCD's L2
    int64_t tm, tn;
    tile_of_block(blockIdx.x, (int64_t)gridDim.x, tiles_m, (n + kHBN - 1) / kHBN, kHGroupM, tm, tn);
    const int64_t m0 = tm * kHBM, n0 = tn * kHBN;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;

    // acc[R][G][r]: the update of C(m0 + 64wm + 16R + li, n0 + 64wn + 16G + 4lg + r)
    f4 acc[4][4];
#pragma unroll
    for (int R = 0; R < 4; ++R)
#pragma unroll
        for (int G = 0; G < 4; ++G) acc[R][G] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t rbase = m0 + 64 * wm + li, cbase = n0 + 64 * wn + 4 * lg;
    const bool inner = m0 + kHBM <= m && n0 + kHBN <= n;  // uniform

    // global -> register staging: A tile 128 x 64 halves = 1024 x 16 B, 4 per thread
    u4 ra[4], rb[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;           // 16-byte unit
            const int row = e >> 3, kk = (e & 7) * 8;
            const int64_t gi = m0 + row, gj = n0 + row;
            ra[q] = (gi < m) ? *(const u4 *)(A16 + blk_index(gi, k0 + kk, sa)) : (u4){0, 0, 0, 0};
            rb[q] = (gj < n) ? *(const u4 *)(B16 + blk_index(gj, k0 + kk, sb)) : (u4){0, 0, 0, 0};
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            const int row = e >> 3, kk = (e & 7) * 8;
            *(u4 *)&As[buf][row][kk] = ra[q];
            *(u4 *)&Bs[buf][row][kk] = rb[q];
        }
    };
    const int nst = (int)(K / kHBK);
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        if (s + 1 < nst) load((int64_t)(s + 1) * kHBK);
#pragma unroll
        for (int kc = 0; kc < kHBK; kc += 32) {
            h8 af[4], bf[4];
#pragma unroll
            for (int R = 0; R < 4; ++R) af[R] = *(const h8 *)&As[buf][64 * wm + 16 * R + li][kc + 8 * lg];
#pragma unroll
            for (int G = 0; G < 4; ++G) bf[G] = *(const h8 *)&Bs[buf][64 * wn + 16 * G + li][kc + 8 * lg];
#pragma unroll
            for (int R = 0; R < 4; ++R)
#pragma unroll
                for (int G = 0; G < 4; ++G) {
                    if constexpr (FMT == 0)
                        acc[R][G] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bf[G], af[R], acc[R][G], 0, 0, 0);
                    else
                        acc[R][G] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[G], af[R], acc[R][G], 0, 0, 0);
                }
        }
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
    }
    // C += acc: an inner tile (all but the last row and column of tiles)
    // reads and writes each column's four rows from one address with
    // immediate offsets; an edge tile tests every element
    if (inner) {
#pragma unroll
        for (int G = 0; G < 4; ++G)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float *col = C + off(rbase, cbase + 16 * G + r, ldc);
#pragma unroll
                for (int R = 0; R < 4; ++R) col[16 * R] += acc[R][G][r];
            }
    } else {
#pragma unroll
        for (int R = 0; R < 4; ++R)
#pragma unroll
            for (int G = 0; G < 4; ++G)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t i = rbase + 16 * R, j = cbase + 16 * G + r;
                    if (i < m && j < n) C[off(i, j, ldc)] += acc[R][G][r];
                }
    }
}

// ---------------------------------------------------------------------------
// The same update on 256 x 128 tiles for the large trailing matrices.  With K
// = NB = 1024 a 128 x 128 tile streams 512 KB of operands through its k-loop,
// and its double-buffered staging leaves each load one 64-k step of matrix-core
// work (~0.2 us) to arrive in: the loop waits on the operands far more than it
// computes.  Here:
//  * tile 256 x 128, 4 waves of 128 x 64 (8 x 4 blocks of 16 x 16, 128 FP32
//    accumulators in AGPRs): a third more matrix-core work per operand byte
//    than the 128 x 128 tile;
//  * K staged 32 at a time (one MFMA k-step) in a ring of 3 LDS buffers of
//    24 KB, filled by global_load_lds_dwordx4 (64 lanes x 16 bytes straight
//    into LDS, no staging registers) two stages ahead; two workgroups per CU,
//    so four stages per CU are in flight while two are computed;
//  * each DMA instruction moves one 1 KB block of the blocked operand layout
//    (16 rows x 32 k, contiguous in memory);
//  * A (and B) sit in LDS as 16-byte units, row r's 4 units (8 k each) in the
//    order s ^ ((r >> 1) & 3): the fragment reads (16 rows x 8 k per lane
//    group) then touch all banks once per 8 lanes.  The DMA takes its swizzle
//    from the lane -> global address map (a permutation within the block);
//  * the accumulators start at zero and C is added once at the end (read into
//    the accumulators up front, C would leave the compiler's waits for those
//    loads inside the k-loop, where -- blind to the DMA of the inline assembly
//    -- they would also drain the stages in flight).
// Requires K % 32 == 0.
// ---------------------------------------------------------------------------
constexpr int kH2M = 256, kH2N = 128, kH2K = 32, kH2S = 3;
constexpr int kH2AInst = kH2M / 16 / 4;  // A DMA instructions per wave per stage (16 rows each)
constexpr int kH2BInst = kH2N / 16 / 4;  // B DMA instructions per wave per stage

#define HPLX_LDS3(p) ((__attribute__((address_space(3))) void *)(p))

template <int FMT>
__global__ __launch_bounds__(256, 2) void hgemm256_update_kernel(int64_t m, int64_t n, int64_t K,
                                                                 const typename Half<FMT>::T *__restrict__ A16,
                                                                 int64_t sa,
                                                                 const typename Half<FMT>::T *__restrict__ B16,
                                                                 int64_t sb, float *__restrict__ C, int64_t ldc,
                                                                 int64_t tiles_m, int64_t tiles_n)
{
    typedef typename Half<FMT>::T H;
    typedef H h8 __attribute__((ext_vector_type(8)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    asm volatile("" ::: "a0");
    __shared__ __attribute__((aligned(1024))) H As[kH2S][kH2M * kH2K];
    __shared__ __attribute__((aligned(1024))) H Bs[kH2S][kH2N * kH2K];
    int64_t tm, tn;
    tile_of_block(blockIdx.x, (int64_t)gridDim.x, tiles_m, tiles_n, 4, tm, tn);
    const int64_t m0 = tm * kH2M, n0 = tn * kH2N;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & 3;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;

    // DMA map: instruction q of an operand stage fills LDS units 64q .. 64q+63;
    // lane i writes unit u = 64q + i = 4r + (s ^ ((r >> 1) & 3)), so it loads
    // row r = 16q + i/4, k segment s = (i & 3) ^ ((r >> 1) & 3): 16 bytes of
    // the block of rows 16q .. 16q+15 of the stage's slab.  Rows (columns)
    // past the matrix are clamped to the last one.
    uint32_t a_off[kH2AInst], b_off[kH2BInst];
#pragma unroll
    for (int q = 0; q < kH2AInst; ++q) {
        const int r = 16 * (kH2AInst * wave + q) + (lane >> 2);
        const int sg = (lane & 3) ^ ((r >> 1) & 3);
        const int64_t rc = (m0 + r < m) ? r : (m - 1 - m0);
        a_off[q] = (uint32_t)((rc >> 4) * 512 + (rc & 15) * 32 + 8 * sg) * 2u;
    }
#pragma unroll
    for (int q = 0; q < kH2BInst; ++q) {
        const int r = 16 * (kH2BInst * wave + q) + (lane >> 2);
        const int sg = (lane & 3) ^ ((r >> 1) & 3);
        const int64_t rc = (n0 + r < n) ? r : (n - 1 - n0);
        b_off[q] = (uint32_t)((rc >> 4) * 512 + (rc & 15) * 32 + 8 * sg) * 2u;
    }
    const char *a_tile = (const char *)(A16 + (size_t)(m0 >> 4) * 512);
    const char *b_tile = (const char *)(B16 + (size_t)(n0 >> 4) * 512);
    const uint32_t lds_a = (uint32_t)(uintptr_t)HPLX_LDS3(&As[0][0]);
    const uint32_t lds_b = (uint32_t)(uintptr_t)HPLX_LDS3(&Bs[0][0]);
    auto dma_stage = [&](int st, int buf) __attribute__((always_inline)) {
        const char *asrc = a_tile + (size_t)st * (size_t)sa * 2;
        const char *bsrc = b_tile + (size_t)st * (size_t)sb * 2;
#pragma unroll
        for (int q = 0; q < kH2AInst; ++q) {
            const uint32_t dst = lds_a + 2u * (uint32_t)(buf * kH2M * kH2K) + 1024u * (uint32_t)(kH2AInst * wave + q);
            asm volatile("global_load_lds_dwordx4 %0, %1" ::"v"(a_off[q]), "s"(asrc), "{m0}"(dst) : "memory");
        }
#pragma unroll
        for (int q = 0; q < kH2BInst; ++q) {
            const uint32_t dst = lds_b + 2u * (uint32_t)(buf * kH2N * kH2K) + 1024u * (uint32_t)(kH2BInst * wave + q);
            asm volatile("global_load_lds_dwordx4 %0, %1" ::"v"(b_off[q]), "s"(bsrc), "{m0}"(dst) : "memory");
        }
    };

    // acc[R][G][r]: the update of C(m0 + 128wm + 16R + li, n0 + 64wn + 16G + 4lg + r)
    f4 acc[8][4];
#pragma unroll
    for (int R = 0; R < 8; ++R)
#pragma unroll
        for (int G = 0; G < 4; ++G) acc[R][G] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t rbase = m0 + 128 * wm + li, cbase = n0 + 64 * wn + 4 * lg;
    const bool inner = m0 + kH2M <= m && n0 + kH2N <= n;  // uniform

    const int nst = (int)(K / kH2K);
    constexpr int kPer = kH2AInst + kH2BInst;  // DMA instructions per wave per stage
    // prologue: stages 0 and 1 in flight; stage 0 landed before the loop
    dma_stage(0, 0);
    if (nst > 1) {
        dma_stage(1, 1);
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kPer) : "memory");
    } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();

    // fragment read offsets (in halves) within a stage buffer
    int a_unit[8], b_unit[4];
#pragma unroll
    for (int R = 0; R < 8; ++R) {
        const int r = 128 * wm + 16 * R + li;
        a_unit[R] = 8 * (4 * r + (lg ^ ((r >> 1) & 3)));
    }
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int c = 64 * wn + 16 * G + li;
        b_unit[G] = 8 * (4 * c + (lg ^ ((c >> 1) & 3)));
    }
    int buf = 0;
    for (int st = 0; st < nst; ++st) {
        if (st + 2 < nst) dma_stage(st + 2, buf == 0 ? 2 : buf - 1);
        h8 af[8], bf[4];
#pragma unroll
        for (int R = 0; R < 8; ++R) af[R] = *(const h8 *)&As[buf][a_unit[R]];
#pragma unroll
        for (int G = 0; G < 4; ++G) bf[G] = *(const h8 *)&Bs[buf][b_unit[G]];
#pragma unroll
        for (int R = 0; R < 8; ++R)
#pragma unroll
            for (int G = 0; G < 4; ++G) {
                if constexpr (FMT == 0)
                    acc[R][G] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bf[G], af[R], acc[R][G], 0, 0, 0);
                else
                    acc[R][G] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[G], af[R], acc[R][G], 0, 0, 0);
            }
        // stage st+1 must have landed; the DMA of stage st+2 may still be in flight
        if (st + 2 < nst)
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kPer) : "memory");
        else
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        buf = (buf == kH2S - 1) ? 0 : buf + 1;
    }

    // C += acc: an inner tile reads and writes each column's 8 rows from one
    // address; an edge tile tests every element
    if (inner) {
#pragma unroll
        for (int G = 0; G < 4; ++G)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float *col = C + off(rbase, cbase + 16 * G + r, ldc);
#pragma unroll
                for (int R = 0; R < 8; ++R) col[16 * R] += acc[R][G][r];
            }
    } else {
#pragma unroll
        for (int G = 0; G < 4; ++G)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = cbase + 16 * G + r;
#pragma unroll
                for (int R = 0; R < 8; ++R)
                    if (j < n && rbase + 16 * R < m) C[off(rbase + 16 * R, j, ldc)] += acc[R][G][r];
            }
    }
}

// ---------------------------------------------------------------------------
// refinement: r = b - A x (FP64, explicit A) in two passes, deterministic:
//   1. workgroup (row block, column chunk q) writes the partial sums
//      P[q][i] = sum_{j in chunk q} a_ij x_j (FMA chain, j in order) and, on
//      the first pass, PA[q][i] = sum_{j in chunk q} |a_ij|;
//   2. one thread per row adds the kResSplit partials in q order, writes
//      r_i = b_i - sum, and the maxima |r_i|, |x_i|, |b_i|, sum_j |a_ij| go to
//      red[0..3] as bit patterns of non-negative doubles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mxp_resid_partial_kernel(const double *__restrict__ A, int64_t lda,
                                                                const double *__restrict__ x, int64_t n,
                                                                int64_t chunk, int anorm, double *__restrict__ P,
                                                                double *__restrict__ PA)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (i >= n) return;
    const int64_t j0 = (int64_t)q * chunk, j1 = (j0 + chunk) < n ? (j0 + chunk) : n;
    double s = 0.0, sa = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double a = A[off(i, j, lda)];
        s = __fma_rn(a, x[j], s);
        if (anorm) sa += fabs(a);
    }
    P[(size_t)q * (size_t)n + i] = s;
    if (anorm) PA[(size_t)q * (size_t)n + i] = sa;
}

__global__ __launch_bounds__(256) void mxp_resid_final_kernel(const double *__restrict__ P,
                                                              const double *__restrict__ PA, int nsplit,
                                                              const double *__restrict__ x,
                                                              const double *__restrict__ b, double *__restrict__ r,
                                                              int64_t n, int anorm,
                                                              unsigned long long *__restrict__ red)
{
    __shared__ double sh[4][4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double vr = 0.0, vx = 0.0, vb = 0.0, va = 0.0;
    if (i < n) {
        double s = 0.0, sa = 0.0;
        for (int q = 0; q < nsplit; ++q) {
            s += P[(size_t)q * (size_t)n + i];
            if (anorm) sa += PA[(size_t)q * (size_t)n + i];
        }
        const double ri = b[i] - s;
        r[i] = ri;
        vr = fabs(ri);
        vx = fabs(x[i]);
        vb = fabs(b[i]);
        va = sa;
    }
    double v[4] = {vr, vx, vb, va};
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int o = 32; o > 0; o >>= 1) v[q] = fmax(v[q], __shfl_xor(v[q], o, 64));
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[threadIdx.x >> 6][q] = v[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int q = threadIdx.x;
        const double mm = fmax(fmax(sh[0][q], sh[1][q]), fmax(sh[2][q], sh[3][q]));
        atomicMax(red + q, (unsigned long long)__double_as_longlong(mm));
    }
}

__global__ __launch_bounds__(256) void axpy_kernel(double *__restrict__ x, const double *__restrict__ d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += d[i];
}

int64_t blocks_of(int64_t n, int64_t per) { return (n + per - 1) / per; }

}  // namespace

int launch_mxp_diag(double *A, int64_t n, int64_t lda, hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    hipLaunchKernelGGL(mxp_diag_kernel, dim3((unsigned)blocks_of(n, 256)), dim3(256), 0, st, A, n, lda);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_cvt_f64_f32(const double *A, int64_t lda, float *B, int64_t ldb, int64_t rows, int64_t cols,
                       hipStream_t st)
{
    if (rows <= 0 || cols <= 0) return HPL_OK;
    const int64_t gx = blocks_of(blocks_of(rows, 2), 256);
    int64_t gy = blocks_of(cols, kCvCols);
    if (gy > 65535) gy = 65535;  // the kernel loops over further column groups
    if (gx > 0x7fffffffll) return HPL_ERR_INTERNAL;
    const bool vec = (lda % 2) == 0 && (ldb % 2) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 8) == 0;
    if (vec)
        hipLaunchKernelGGL(cvt_f64_f32_kernel<true>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, A, lda, B,
                           ldb, rows, cols);
    else
        hipLaunchKernelGGL(cvt_f64_f32_kernel<false>, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, A, lda, B,
                           ldb, rows, cols);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_panel32_leaf(float *A, int64_t lda, int64_t c, int64_t n, int w, unsigned long long *info,
                        unsigned *done, hipStream_t st, unsigned *mx, int64_t l21_row0)
{
    if (w <= 0 || w > kPanel32LeafMax) return HPL_ERR_INTERNAL;
    const int64_t below = n - c - w;
    const int lw = w <= 32 ? 32 : 64;
    const int64_t g = below > 0 ? blocks_of(below, 256 - lw) : 1;
    if (g > 0xffffffffll) return HPL_ERR_INTERNAL;
    if (lw == 32)
        hipLaunchKernelGGL(panel32_leaf_kernel<32>, dim3((unsigned)g), dim3(256), 0, st, A, lda, c, n, w, info, done,
                           mx, l21_row0);
    else
        hipLaunchKernelGGL(panel32_leaf_kernel<64>, dim3((unsigned)g), dim3(256), 0, st, A, lda, c, n, w, info, done,
                           mx, l21_row0);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_trsm32_leaf(const float *L, int64_t ldl, float *B, int64_t ldb, int nbk, int64_t ncols, hipStream_t st,
                       unsigned *mx)
{
    if (ncols <= 0 || nbk <= 0) return HPL_OK;
    if (nbk > kTrsm32LeafMax) return HPL_ERR_INTERNAL;
    const int64_t g = blocks_of(ncols, kTlCols);
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    // 16-byte vectors need every column start 16-byte aligned and all rows present
    const bool al = ((uintptr_t)B % 16) == 0 && (ldb % 4) == 0;
    if (nbk <= 32) {
        if (nbk == 32 && al)
            hipLaunchKernelGGL((trsm32_leaf_kernel<32, true>), dim3((unsigned)g), dim3(kTlCols), 0, st, L, ldl, B, ldb,
                               nbk, ncols, mx);
        else
            hipLaunchKernelGGL((trsm32_leaf_kernel<32, false>), dim3((unsigned)g), dim3(kTlCols), 0, st, L, ldl, B,
                               ldb, nbk, ncols, mx);
    } else {
        if (nbk == 64 && al)
            hipLaunchKernelGGL((trsm32_leaf_kernel<64, true>), dim3((unsigned)g), dim3(kTlCols), 0, st, L, ldl, B, ldb,
                               nbk, ncols, mx);
        else
            hipLaunchKernelGGL((trsm32_leaf_kernel<64, false>), dim3((unsigned)g), dim3(kTlCols), 0, st, L, ldl, B,
                               ldb, nbk, ncols, mx);
    }
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_sgemm32(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B, int64_t ldb,
                   float *C, int64_t ldc, hipStream_t st)
{
    if (m <= 0 || n <= 0 || k <= 0) return HPL_OK;
    const int64_t gx = blocks_of(m, 64), gy = blocks_of(n, 64);
    if (gy > 65535) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(sgemm32_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, m, n, k, A, lda, B, ldb,
                       C, ldc);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_mxp_convert(int fmt, const float *L, int64_t ldl, int64_t m, const float *U, int64_t ldu, int64_t ncols,
                       int w, const unsigned *mx, unsigned *reset, void *A16, int64_t sa, void *B16, int64_t sb,
                       hipStream_t st)
{
    if (w % 32 || sa % 512 || sb % 512) return HPL_ERR_INTERNAL;
    const int64_t gl = blocks_of(m, 64), gk = blocks_of(w, 64);
    const int64_t gu = blocks_of((int64_t)(w / 32) * blocks_of(ncols, 16) * 512, 256);
    const int64_t g = gl * gk + gu;
    if (g < 1 || g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    if (fmt == 0)
        hipLaunchKernelGGL(cvt_lu_kernel<0>, dim3((unsigned)g), dim3(256), 0, st, L, ldl, m, w, U, ldu, ncols, mx,
                           reset, (_Float16 *)A16, sa, (_Float16 *)B16, sb, gl, gk);
    else
        hipLaunchKernelGGL(cvt_lu_kernel<1>, dim3((unsigned)g), dim3(256), 0, st, L, ldl, m, w, U, ldu, ncols, mx,
                           reset, (__bf16 *)A16, sa, (__bf16 *)B16, sb, gl, gk);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_hgemm_update(int fmt, int64_t m, int64_t n, int64_t K, const void *A16, int64_t sa, const void *B16,
                        int64_t sb, float *C, int64_t ldc, hipStream_t st)
{
    if (m <= 0 || n <= 0 || K <= 0) return HPL_OK;
    if (K % kHBK || sa % 512 || sb % 512) return HPL_ERR_INTERNAL;
    // large updates on 256 x 128 tiles (at least two tiles per CU), the rest
    // on 128 x 128; an element gets the same bits from either
    const int64_t t2m = blocks_of(m, kH2M), t2n = blocks_of(n, kH2N);
    if (t2m * t2n >= 512 && K % kH2K == 0) {
        const int64_t g2 = t2m * t2n;
        if (g2 > 0x7fffffffll) return HPL_ERR_INTERNAL;
        if (fmt == 0)
            hipLaunchKernelGGL(hgemm256_update_kernel<0>, dim3((unsigned)g2), dim3(256), 0, st, m, n, K,
                               (const _Float16 *)A16, sa, (const _Float16 *)B16, sb, C, ldc, t2m, t2n);
        else
            hipLaunchKernelGGL(hgemm256_update_kernel<1>, dim3((unsigned)g2), dim3(256), 0, st, m, n, K,
                               (const __bf16 *)A16, sa, (const __bf16 *)B16, sb, C, ldc, t2m, t2n);
        HPLX_TRY_LAUNCH();
        return HPL_OK;
    }
    const int64_t tiles_m = blocks_of(m, kHBM), tiles_n = blocks_of(n, kHBN);
    const int64_t g = tiles_m * tiles_n;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    if (fmt == 0)
        hipLaunchKernelGGL(hgemm_update_kernel<0>, dim3((unsigned)g), dim3(256), 0, st, m, n, K,
                           (const _Float16 *)A16, sa, (const _Float16 *)B16, sb, C, ldc, tiles_m);
    else
        hipLaunchKernelGGL(hgemm_update_kernel<1>, dim3((unsigned)g), dim3(256), 0, st, m, n, K,
                           (const __bf16 *)A16, sa, (const __bf16 *)B16, sb, C, ldc, tiles_m);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_mxp_residual(const double *A, int64_t lda, const double *x, const double *b, double *r, int64_t n,
                        bool anorm, double *part, unsigned long long *red, hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    const int64_t chunk = (n + kResSplit - 1) / kResSplit;
    double *P = part, *PA = part + (size_t)kResSplit * (size_t)n;
    hipLaunchKernelGGL(mxp_resid_partial_kernel, dim3((unsigned)blocks_of(n, 256), kResSplit), dim3(256), 0, st, A,
                       lda, x, n, chunk, anorm ? 1 : 0, P, PA);
    HPLX_TRY_LAUNCH();
    hipLaunchKernelGGL(mxp_resid_final_kernel, dim3((unsigned)blocks_of(n, 256)), dim3(256), 0, st, P, PA, kResSplit,
                       x, b, r, n, anorm ? 1 : 0, red);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_axpy(double *x, const double *d, int64_t n, hipStream_t st)
{
    if (n <= 0) return HPL_OK;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)blocks_of(n, 256)), dim3(256), 0, st, x, d, n);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
