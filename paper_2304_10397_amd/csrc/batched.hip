// batched.hip -- many independent small dense systems A_i X_i = B_i (n_i <= 512)
// in ONE persistent launch: LU with partial pivoting (the method of Sec. II
// applied to each system: panel FACT, interchanges, U12 = L11^{-1} A12, rank-NB
// trailing update), the solve, and optionally the adjoint of the solve
// (grad_B = A^{-T} W, grad_A = -grad_B X^T) for a loss whose gradient with
// respect to X is W.
//
// Layout (all packed, column-major, leading dimension n_i): A_i at
// aoff_i = sum_{j<i} n_j^2; B_i, X_i, W_i and grad_B_i at nrhs * voff_i, with
// voff_i = sum_{j<i} n_j; ipiv_i at voff_i (0-based within the system,
// sequential-interchange semantics, LAPACK form of L: P A = L U).
//
// Scheduling: 256 persistent workgroups of 512 threads (one per CU; 8 waves,
// 2 per SIMD); each takes the next system from an atomic counter over a
// largest-first order, so the n^3-heavy systems start first and the small
// ones fill the tail.  A system's matrix stays in global memory (L2 / MALL
// resident at these sizes); per 32-column panel step:
//   1. FACT: thread t holds row k0+t of the panel in registers; per column one
//      barrier: each wave publishes its best candidate (|a|, row) and that
//      row's values in LDS (double-buffered by column parity), the diagonal
//      row is published too, and every thread then knows the pivot row and
//      performs the interchange and the rank-1 update of its own row.  The
//      column loop is rolled (the register row rotates by one column per step).
//   2. The 32 interchanges are composed (by one wave, after the column loop) into one
//      permutation of the <= 64 rows they touch; every other column (left:
//      LAPACK-form L; right: U12 and the trailing columns; the right-hand
//      sides, carried as extra columns so that B becomes L^{-1} P B as in
//      HPL's augmented system) goes through LDS in chunks of 64 columns:
//      gathered with lane = slot (the panel rows of a column are consecutive,
//      so the reads coalesce), the right columns' top 32 rows multiplied by
//      L11^{-1} (the triangular inverse, formed once per panel by
//      substitution) on the matrix cores, and scattered to the destination
//      rows.
//   3. Trailing update C -= L21 U12 over rows [k0+32, n) and columns
//      [k0+32, n+nrhs) on the FP64 matrix cores (16 x 16 blocks, masked at
//      the ragged edges), -L21 fragments in registers, U12 through LDS.
// Then U X = Y by 32-row blocks from the bottom.  The adjoint: U^T z = W by
// blocks from the top, L^T v = z from the bottom, grad_B = P^T v (a scatter
// through the row permutation tracked during FACT), grad_A = -grad_B X^T.
// Every wave of every workgroup reaches the queue's exit test, so the grid
// drains when the counter passes the batch size.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kBT = 512;               // threads per workgroup
constexpr int kBW = kBT / 64;          // waves
constexpr int kPBmax = 32;             // widest panel of any variant
constexpr int kSB = 32;                // row block of the solves and the adjoint
constexpr int kKC = 8;                 // right-hand sides per LDS stage of the adjoint
constexpr int kUpdRows = 4;            // 16-row blocks per wave in the trailing update (8 waves x 4 x 16 >= 480)
constexpr int kUCmax = 128;            // widest U12 stage of any variant
constexpr int kGc = 64;                // columns per chunk of the interchange pass

// Variants of the factorization (panel width PB, columns of U12 per LDS stage
// UC); the tuner's table names them by index.
constexpr int kNumVariants = 4;
constexpr int kVarPB[kNumVariants] = {32, 32, 16, 16};
constexpr int kVarUC[kNumVariants] = {128, 64, 128, 64};
static_assert(kNumVariants == HPL_BATCH_VARIANTS, "variant count");

struct BatchArgs {
    int64_t count;
    const int32_t *sizes;  // [count]
    const int64_t *aoff;   // [count] element offset of A_i
    const int64_t *voff;   // [count] sum of the preceding sizes
    const int32_t *order;  // [count] processing order (largest first)
    double *A;
    int32_t *ipiv;
    double *B;
    const double *W;
    double *GB;
    double *GA;
    int nrhs;
    int mode;              // bit 0: factor + solve; bit 1: adjoint
    int64_t *info;         // [count]
    unsigned *counter;     // zero before the launch
    signed char vtab[kBatchBuckets];  // variant of each size bucket (n - 1) / 32
};

struct BatchShared {
    union {
        double Lc[kKC][kBatchMaxN];                // right-hand-side stage of the adjoint
        double G32[kGc][2 * 32 + 1];               // interchange pass: [column][slot], PB = 32
        double G16[kGc][2 * 16 + 1];               // ... PB = 16
        double Us32x128[32][128 + 8];              // trailing update: U12 [k][column], per (PB, UC)
        double Us32x64[32][64 + 8];
        double Us16x128[16][128 + 8];
        double Us16x64[16][64 + 8];
    };
    double T[kPBmax][kPBmax + 1];          // diagonal block (L11, or a block of U / L for the solves)
    double Ti[kPBmax][kPBmax + 1];         // L11^{-1}, identity past the panel width
    double Ur[kPBmax][kPBmax];             // the panel's pivot rows, step j: slot q = column k0+j+q
    double pv[kBW];                        // per-wave candidate |a|
    int pr[kBW];                           // per-wave candidate (logical) row
    double Ys[kBatchMaxRhs][kSB];          // solved block of the solves
    int perm[kBatchMaxN];                  // row permutation: row i of P A is row perm[i] of A
    int slot_row[2 * kPBmax];              // interchange composition: destination rows ...
    int slot_src[2 * kPBmax];              // ... and the original row each receives
    int pivs[kPBmax];                      // the panel's pivot rows, in column order
    int nslots;
    int64_t info;
    int64_t job;
};

// global-memory pointers for the phase functions (a plain pointer argument of a
// non-inlined function is generic, and generic accesses share the LDS wait
// counter)
typedef __attribute__((address_space(1))) double gf64;
typedef __attribute__((address_space(1))) const double gcf64;
typedef __attribute__((address_space(1))) int32_t gi32;

// the workgroup's shared state (one workgroup per CU; file scope, so that the
// phase functions below address it as LDS without a pointer argument)
__shared__ BatchShared sh;

// the interchange stage and the U12 stage of a variant
template <int PB>
__device__ __forceinline__ double &gstage(int c, int slot)
{
    if constexpr (PB == 32) return sh.G32[c][slot];
    else return sh.G16[c][slot];
}

template <int PB, int UC>
__device__ __forceinline__ double &ustage(int k, int j)
{
    if constexpr (PB == 32 && UC == 128) return sh.Us32x128[k][j];
    else if constexpr (PB == 32) return sh.Us32x64[k][j];
    else if constexpr (UC == 128) return sh.Us16x128[k][j];
    else return sh.Us16x64[k][j];
}

__device__ __forceinline__ gf64 *col_ptr(gf64 *a, gf64 *b, int n, int c)
{
    return c < n ? a + (size_t)c * (size_t)n : b + (size_t)(c - n) * (size_t)n;
}


// FACT of the panel [k0, k0+w) (rows k0..n-1 in registers), its interchanges
// recorded in ip, the permutation and the slot lists; L11 left in sh.T.
// Rows do not move between threads: thread t holds row k0+t as loaded and the
// logical row lr that row has become (an interchange swaps two lr values).
// Step j's column is always v[0]: the rank-1 update writes slot q's result
// into slot q-1 and the column's multiplier into the last slot, so the loop
// is not unrolled and every register index is a constant.  Only the winning
// row is published (into sh.Ur[j], its finished slots zeroed): a zero u
// leaves a row's finished slots -- its earlier multipliers -- unchanged, so
// the update needs no per-slot masks.
template <int PB, int OCC>
__device__ __attribute__((noinline)) void bat_panel(gf64 *a, gi32 *ip, int n, int k0)
{
    constexpr int kPB = PB;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int w = (n - k0) < kPB ? (n - k0) : kPB;
    const int r = k0 + t;
    const bool own = r < n;
    // the panel rows, all loads issued at once: a row past the system (not
    // own) or a column past the panel (q >= w) reads a clamped element that
    // is never used -- masking it would put each load behind a branch that
    // waits for it
    double v[kPB];
    {
        const int rr = own ? r : n - 1;
#pragma unroll
        for (int q = 0; q < kPB; ++q) {
            const int cq = (k0 + q) < n ? (k0 + q) : (n - 1);
            v[q] = a[(size_t)rr + (size_t)cq * (size_t)n];
        }
    }
    int lr = r;
    __syncthreads();
    for (int j = 0; j < w; ++j) {
        const int kj = k0 + j;
        // wave argmax of |v[0]| over logical rows >= k0+j (a NaN ranks below
        // every number); ties: the lowest logical row
        const double av = fabs(v[0]);
        const double cv = (own && lr >= kj) ? (av == av ? av : -0.5) : -1.0;
        const double vm = wave_max(cv);
        const unsigned rm = wave_min_u32(cv == vm ? (unsigned)lr : 0xffffffffu);
        if (lane == 0) {
            sh.pv[wave] = vm;
            sh.pr[wave] = (int)rm;
        }
        __syncthreads();
        // the winner over the waves (a wave without candidates reports -1)
        const double x = lane < kBW ? sh.pv[lane] : -2.0;
        const unsigned y = lane < kBW ? (unsigned)sh.pr[lane] : 0xffffffffu;
        const double gv = wave_max(x);
        const int gp = (int)wave_min_u32(x == gv ? y : 0xffffffffu);
        // its thread publishes the row: slots of the panel's remaining
        // columns, zeros past them
        if (own && lr == gp) {
#pragma unroll
            for (int q = 0; q < kPB; ++q) sh.Ur[j][q] = q < w - j ? v[q] : 0.0;
        }
        if (t == 0) sh.pivs[j] = gp;  // composed after the loop (off the per-column path)
        __syncthreads();
        double u[kPB];
#pragma unroll
        for (int q = 0; q < kPB; ++q) u[q] = sh.Ur[j][q];
        // the interchange of logical rows k0+j and gp
        if (lr == kj)
            lr = gp;
        else if (lr == gp)
            lr = kj;
        const double piv = u[0];
        const bool sing = piv == 0.0;  // column left unscaled, no update
        if (sing && t == 0 && sh.info == 0) sh.info = kj + 1;
        const double l = sing ? v[0] : v[0] / piv;
        const double lu = (own && lr > kj && !sing) ? l : 0.0;
#pragma unroll
        for (int q = 1; q < kPB; ++q) v[q - 1] = __fma_rn(-lu, u[q], v[q]);
        v[kPB - 1] = l;
    }
    // w steps so far: rotate the rest of the turn, so that slot q holds the
    // multiplier of column k0+q
    for (int j = w; j < kPB; ++j) {
        const double c0 = v[0];
#pragma unroll
        for (int q = 0; q < kPB - 1; ++q) v[q] = v[q + 1];
        v[kPB - 1] = c0;
    }
    // the panel's interchanges composed by wave 0: lane j follows destination
    // row k0+j (and, if it is the first occurrence of a pivot row below the
    // panel, that row) back through the transpositions, last first, to the
    // original row it receives; the row permutation and the slot lists of the
    // interchange pass follow, and ipiv is written
    __syncthreads();
    if (wave == 0) {
        int g[kPB];
#pragma unroll
        for (int q = 0; q < kPB; ++q) g[q] = q < w ? sh.pivs[q] : -1;
        const int j = lane;
        int gj = -1;
#pragma unroll
        for (int q = 0; q < kPB; ++q)
            if (q == j) gj = g[q];
        bool isx = j < w && gj >= k0 + w;
#pragma unroll
        for (int q = 0; q < kPB; ++q)
            if (q < j && g[q] == gj) isx = false;
        const unsigned long long bx = __ballot(isx);
        const int nx = __popcll(bx);
        const int xi = __popcll(bx & ((1ull << j) - 1ull));
        auto sigma = [&](int d) {
#pragma unroll
            for (int q = kPB - 1; q >= 0; --q)
                if (q < w) {
                    if (d == k0 + q)
                        d = g[q];
                    else if (d == g[q])
                        d = k0 + q;
                }
            return d;
        };
        const int d0 = k0 + (j < w ? j : 0), s0 = sigma(d0);
        const int dx = isx ? gj : d0, sx = sigma(dx);
        const int p0 = sh.perm[s0], px = sh.perm[sx];  // every read before any write
        if (j < w) {
            sh.slot_row[j] = d0;
            sh.slot_src[j] = s0;
            ip[k0 + j] = gj;
        }
        if (isx) {
            sh.slot_row[w + xi] = dx;
            sh.slot_src[w + xi] = sx;
        }
        if (j == 0) sh.nslots = w + nx;
        if (j < w) sh.perm[d0] = p0;
        if (isx) sh.perm[dx] = px;
    }
    // write the factored panel back: each row's multipliers to its logical
    // row (a row of U11 holds those left of its diagonal), the rows of U from
    // sh.Ur; L11 and U11 to sh.T
    if (own) {
        const int nl = lr < k0 + w ? lr - k0 : w;
#pragma unroll
        for (int q = 0; q < kPB; ++q)
            if (q < nl) a[(size_t)lr + (size_t)(k0 + q) * (size_t)n] = v[q];
        if (lr < k0 + w) {
#pragma unroll
            for (int q = 0; q < kPB; ++q)
                if (q < nl) sh.T[lr - k0][q] = v[q];
        }
    }
    if (t < w) {
#pragma unroll
        for (int q = 0; q < kPB; ++q)
            if (q >= t && q < w) {
                const double x = sh.Ur[t][q - t];
                sh.T[t][q] = x;
                a[(size_t)(k0 + t) + (size_t)(k0 + q) * (size_t)n] = x;
            }
    }
    __syncthreads();
}

template <int PB, int OCC>
__device__ __attribute__((noinline)) void bat_interchange(gf64 *a, gf64 *b, int n, int ncol, int k0, int w)
{
    constexpr int kPB = PB, kMaxSlots = 2 * PB;
    constexpr int kGq = kGc * kMaxSlots / kBT;  // gathered values per thread and chunk
    static_assert(kBT % kMaxSlots == 0 && kGc % (kBT / kMaxSlots) == 0, "interchange pass shape");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nslots = sh.nslots;
    const int nother = ncol - w;
    const int slot = t & (kMaxSlots - 1), cq = t / kMaxSlots;  // kBT / kMaxSlots columns per pass
    const int src = sh.slot_src[slot < nslots ? slot : nslots - 1];
    const int dst = sh.slot_row[slot < nslots ? slot : nslots - 1];
    // the gather of a chunk of kGc columns (lane = slot, so the panel rows of
    // a column are read coalesced); issued one chunk ahead, so that its loads
    // are in flight while the previous chunk is multiplied and scattered
    double gq[kGq];
    auto gather = [&](int e0) __attribute__((always_inline)) {
        const int ce = (nother - e0) < kGc ? (nother - e0) : kGc;
#pragma unroll
        for (int q = 0; q < kGq; ++q) {
            const int cl = cq + q * (kBT / kMaxSlots);
            const int e = e0 + (cl < ce ? cl : ce - 1);
            const int c = e < k0 ? e : e + w;
            gq[q] = col_ptr(a, b, n, c)[src];
        }
    };
    if (nother > 0) gather(0);
    // ---- 1. L11^{-1} (the triangular inverse; unit lower, identity past the
    //      panel width) into sh.Ti: lane j of wave 0 solves L11 y = e_j row by
    //      row, y_i = -sum_{k<i} l_ik y_k, with y_k = 0 above the diagonal
    if (wave == 0 && lane < kPB) {
        double y[kPB];
#pragma unroll
        for (int i = 0; i < kPB; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) acc = __fma_rn(-sh.T[i][k], y[k], acc);
            y[i] = (i == lane) ? 1.0 : ((i > lane && i < w) ? acc : 0.0);
        }
#pragma unroll
        for (int i = 0; i < kPB; ++i) sh.Ti[i][lane] = y[i];
    }
    // ---- 2. interchanges on every other column; U12 = L11^{-1} A12 on the right.
    //      Chunks of kGc columns through LDS: gathered, the right columns' top
    //      rows multiplied by L11^{-1} on the matrix cores (one 16 x 16 block
    //      per wave), scattered.
    {
        for (int e0 = 0; e0 < nother; e0 += kGc) {
            const int ce = (nother - e0) < kGc ? (nother - e0) : kGc;
#pragma unroll
            for (int q = 0; q < kGq; ++q) {
                const int cl = cq + q * (kBT / kMaxSlots);
                gstage<PB>(cl, slot) = gq[q];
            }
            __syncthreads();
            if (e0 + kGc < nother) gather(e0 + kGc);
            if (e0 + ce > k0) {  // the chunk has right columns (uniform)
                // block (rb, cb) of Y = L11^{-1} G_top: rows 16 rb.., columns 16 cb..;
                // lane l supplies Ti(16 rb + l%16, 4 s + l/16) and G(4 s + l/16, 16 cb + l%16)
                typedef double d4 __attribute__((ext_vector_type(4)));
                constexpr int kRB = kPB / 16, kCB = kGc / 16;
                const int rb = wave % kRB, cb = wave / kRB;
                const int li = lane & 15, lg = lane >> 4;
                d4 y = {0.0, 0.0, 0.0, 0.0};
                if (cb < kCB) {
#pragma unroll
                    for (int s4 = 0; s4 < kPB / 4; ++s4)
                        y = __builtin_amdgcn_mfma_f64_16x16x4f64(sh.Ti[16 * rb + li][4 * s4 + lg],
                                                                 gstage<PB>(16 * cb + li, 4 * s4 + lg), y, 0, 0, 0);
                }
                __syncthreads();  // every fragment of G read before any is replaced
                if (cb < kCB) {
                    const int cl = 16 * cb + li;
                    if (cl < ce && e0 + cl >= k0) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) gstage<PB>(cl, 16 * rb + lg + 4 * r) = y[r];
                    }
                }
            }
            __syncthreads();
            if (slot < nslots) {
#pragma unroll
                for (int q = 0; q < kGq; ++q) {
                    const int cl = cq + q * (kBT / kMaxSlots);
                    if (cl < ce) {
                        const int e = e0 + cl;
                        const int c = e < k0 ? e : e + w;
                        col_ptr(a, b, n, c)[dst] = gstage<PB>(cl, slot);
                    }
                }
            }
            __syncthreads();
        }
    }

}

// Trailing update C -= L21 U12 (rows and columns from k0+32; the last panel,
// narrower than 32, leaves no trailing matrix) on the FP64 matrix cores:
// 16 x 16 blocks, v_mfma_f64_16x16x4_f64, K = 32 as 8 MFMAs.  Wave w owns
// block-rows w, w+8, ..; its -L21 fragments (lane l: row 16R + l%16, k = 4s +
// l/16) stay in registers for the whole step; U12 goes through LDS 128
// columns at a time.  The U fragment is the MFMA's first operand, so a block
// comes out transposed: register r of lane l is C(16R + l%16, 16G + l/16 +
// 4r), 16 consecutive rows per access.  Accumulators start from C; the
// products are added in k order.
template <int PB, int UC, int OCC>
__device__ __attribute__((noinline)) void bat_update(gf64 *a, gf64 *b, int n, int ncol, int k0, int w)
{
    constexpr int kPB = PB, kUpdCols = UC;
    typedef double d4 __attribute__((ext_vector_type(4)));
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int r0 = k0 + w;
    const int m = n - r0, nc = ncol - r0;
    if (m <= 0 || nc <= 0 || w != kPB) return;
    const int nR = (m + 15) >> 4, nG = (nc + 15) >> 4;
    double af[kUpdRows][kPB / 4];
#pragma unroll
    for (int q = 0; q < kUpdRows; ++q) {
        const int row = r0 + 16 * (wave + kBW * q) + li;
        const bool ok = (wave + kBW * q) < nR && row < n;
        const int rc = row < n ? row : n - 1;
#pragma unroll
        for (int s4 = 0; s4 < kPB / 4; ++s4) {
            const double x = a[(size_t)rc + (size_t)(k0 + 4 * s4 + lg) * (size_t)n];
            af[q][s4] = ok ? -x : 0.0;
        }
    }
    for (int cc0 = 0; cc0 < nc; cc0 += kUpdCols) {
        // stage U12[:, cc0 .. cc0+128) as Us[k][j] (burst: 8 loads per thread)
        {
            constexpr int kQ = kPB * kUpdCols / kBT;
            double uq[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = t + q * kBT, k = e % kPB, jj = e / kPB;
                const int jc = (cc0 + jj) < nc ? (cc0 + jj) : (nc - 1);
                const double x = col_ptr(a, b, n, r0 + jc)[k0 + k];
                uq[q] = (cc0 + jj) < nc ? x : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = t + q * kBT;
                ustage<PB, UC>(e % kPB, e / kPB) = uq[q];
            }
        }
        __syncthreads();
        const int g0 = cc0 >> 4;
        const int gn = (nG - g0) < (kUpdCols / 16) ? (nG - g0) : (kUpdCols / 16);
        // per row block: the C values of all the stage's column blocks are
        // loaded at once (clamped addresses, so no load waits on a branch),
        // then each live block takes its MFMAs and is stored
        constexpr int kGB = kUpdCols / 16;
#pragma unroll
        for (int q = 0; q < kUpdRows; ++q) {
            const int R = wave + kBW * q;
            if (R < nR) {
                const int row = r0 + 16 * R + li;
                const int rc = row < n ? row : n - 1;
                d4 cv[kGB];
#pragma unroll
                for (int g = 0; g < kGB; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int c = r0 + 16 * (g0 + g) + lg + 4 * r;
                        cv[g][r] = col_ptr(a, b, n, c < ncol ? c : ncol - 1)[rc];
                    }
                // the store addresses are recomputed from a laundered copy of the
                // stage's first column (so they are not kept live from the loads)
                int c0s = r0 + 16 * g0;
                asm volatile("" : "+v"(c0s));
#pragma unroll
                for (int g = 0; g < kGB; ++g) {
                    if (g < gn) {
#pragma unroll
                        for (int s4 = 0; s4 < kPB / 4; ++s4) {
                            const double bu = ustage<PB, UC>(4 * s4 + lg, 16 * g + li);
                            cv[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(bu, af[q][s4], cv[g], 0, 0, 0);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int c = c0s + 16 * g + lg + 4 * r;
                            if (c < ncol && row < n) col_ptr(a, b, n, c)[row] = cv[g][r];
                        }
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // one row block's C in registers at a time
        }
        __syncthreads();
    }
}

// U X = Y, 32-row blocks from the bottom (Y = L^{-1} P B is in b)
template <int OCC>
__device__ __attribute__((noinline)) void bat_usolve(gcf64 *a, gf64 *b, int n, int nrhs)
{
    constexpr int kPB = OCC == 2 ? 16 : kSB;  // a narrower block keeps two systems per CU within 128 VGPRs
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nb0 = (n - 1) / kPB * kPB;
    for (int r0 = nb0; r0 >= 0; r0 -= kPB) {
        const int bw = (n - r0) < kPB ? (n - r0) : kPB;
        {
            constexpr int kTQ = (kPB * kPB + kBT - 1) / kBT;
            double tq[kTQ];
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int ee = t + q * kBT, e = ee < kPB * kPB ? ee : kPB * kPB - 1, i = e % kPB, k = e / kPB;
                const int ic = i < bw ? i : bw - 1, kc = k < bw ? k : bw - 1;
                tq[q] = a[(size_t)(r0 + ic) + (size_t)(r0 + kc) * (size_t)n];
            }
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int e = t + q * kBT;
                if (e < kPB * kPB) sh.T[e % kPB][e / kPB] = tq[q];
            }
        }
        __syncthreads();
        for (int rh = wave; rh < nrhs; rh += kBW) {
            gf64 *bp = b + (size_t)rh * (size_t)n;
            double y = bp[r0 + (lane < bw ? lane : bw - 1)];
            for (int s = bw - 1; s >= 0; --s) {
                const double xs = read_lane(y, s) / sh.T[s][s];
                if (lane == s) y = xs;
                if (lane < s) y = __fma_rn(-sh.T[lane][s], xs, y);
            }
            if (lane < bw) {
                bp[r0 + lane] = y;
                sh.Ys[rh][lane] = y;
            }
        }
        __syncthreads();
        for (int i = t; i < r0; i += kBT) {
            double u[kPB];
#pragma unroll
            for (int k = 0; k < kPB; ++k) {
                const int kc = k < bw ? k : bw - 1;
                u[k] = a[(size_t)i + (size_t)(r0 + kc) * (size_t)n];
            }
            for (int rh = 0; rh < nrhs; ++rh) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < kPB; ++k)
                    if (k < bw) acc = __fma_rn(u[k], sh.Ys[rh][k], acc);
                gf64 *bp = b + (size_t)rh * (size_t)n;
                bp[i] = bp[i] - acc;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// forward: LU with partial pivoting of the augmented [A | B], then U X = Y
// ---------------------------------------------------------------------------
template <int PB, int UC, int OCC>
__device__ void batch_forward(double *a, double *b, int32_t *ip, int n, int nrhs)
{
    constexpr int kPB = PB;
    const int t = threadIdx.x;
    const int ncol = n + nrhs;
    for (int i = t; i < n; i += kBT) sh.perm[i] = i;
    if (t == 0) sh.info = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += kPB) {
        const int w = (n - k0) < kPB ? (n - k0) : kPB;
        bat_panel<PB, OCC>((gf64 *)a, (gi32 *)ip, n, k0);
        bat_interchange<PB, OCC>((gf64 *)a, (gf64 *)b, n, ncol, k0, w);
        bat_update<PB, UC, OCC>((gf64 *)a, (gf64 *)b, n, ncol, k0, w);
    }
    bat_usolve<OCC>((gcf64 *)a, (gf64 *)b, n, nrhs);
}

// ---------------------------------------------------------------------------
// adjoint: grad_B = A^{-T} W = P^T L^{-T} U^{-T} W, grad_A = -grad_B X^T
// ---------------------------------------------------------------------------
template <int OCC>
__device__ __attribute__((noinline)) void batch_adjoint(gcf64 *a, gcf64 *x, gcf64 *wv, gf64 *gb,
                              gf64 *ga, int n, int nrhs)
{
    constexpr int kPB = OCC == 2 ? 16 : kSB;  // a narrower block keeps two systems per CU within 128 VGPRs
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    {
        constexpr int kQ = kBatchMaxN * kBatchMaxRhs / kBT;
        double wq[kQ];
        const int tot = n * nrhs;
#pragma unroll
        for (int q = 0; q < kQ; ++q) wq[q] = wv[(t + q * kBT) < tot ? (t + q * kBT) : tot - 1];
#pragma unroll
        for (int q = 0; q < kQ; ++q)
            if (t + q * kBT < tot) gb[t + q * kBT] = wq[q];
    }
    __syncthreads();
    // U^T z = W: lower with diagonal u_ii, blocks from the top
    for (int r0 = 0; r0 < n; r0 += kPB) {
        const int bw = (n - r0) < kPB ? (n - r0) : kPB;
        {
            constexpr int kTQ = (kPB * kPB + kBT - 1) / kBT;
            double tq[kTQ];
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int ee = t + q * kBT, e = ee < kPB * kPB ? ee : kPB * kPB - 1, i = e % kPB, k = e / kPB;
                const int ic = i < bw ? i : bw - 1, kc = k < bw ? k : bw - 1;
                tq[q] = a[(size_t)(r0 + ic) + (size_t)(r0 + kc) * (size_t)n];
            }
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int e = t + q * kBT;
                if (e < kPB * kPB) sh.T[e % kPB][e / kPB] = tq[q];
            }
        }
        __syncthreads();
        for (int rh = wave; rh < nrhs; rh += kBW) {
            gf64 *zp = gb + (size_t)rh * (size_t)n;
            double y = zp[r0 + (lane < bw ? lane : bw - 1)];
            for (int s = 0; s < bw; ++s) {
                const double xs = read_lane(y, s) / sh.T[s][s];
                if (lane == s) y = xs;
                if (lane > s && lane < bw) y = __fma_rn(-sh.T[s][lane], xs, y);  // U^T(lane, s) = U(s, lane)
            }
            if (lane < bw) {
                zp[r0 + lane] = y;
                sh.Ys[rh][lane] = y;
            }
        }
        __syncthreads();
        for (int i = r0 + bw + t; i < n; i += kBT) {
            double u[kPB];  // U(r0 + k, i): column i, contiguous
#pragma unroll
            for (int k = 0; k < kPB; ++k) u[k] = a[(size_t)(r0 + (k < bw ? k : bw - 1)) + (size_t)i * (size_t)n];
            for (int rh = 0; rh < nrhs; ++rh) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < kPB; ++k)
                    if (k < bw) acc = __fma_rn(u[k], sh.Ys[rh][k], acc);
                gf64 *zp = gb + (size_t)rh * (size_t)n;
                zp[i] = zp[i] - acc;
            }
        }
        __syncthreads();
    }
    // L^T v = z: unit upper, blocks from the bottom
    const int nb0 = (n - 1) / kPB * kPB;
    for (int r0 = nb0; r0 >= 0; r0 -= kPB) {
        const int bw = (n - r0) < kPB ? (n - r0) : kPB;
        {
            constexpr int kTQ = (kPB * kPB + kBT - 1) / kBT;
            double tq[kTQ];
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int ee = t + q * kBT, e = ee < kPB * kPB ? ee : kPB * kPB - 1, i = e % kPB, k = e / kPB;
                const int ic = i < bw ? i : bw - 1, kc = k < bw ? k : bw - 1;
                tq[q] = a[(size_t)(r0 + ic) + (size_t)(r0 + kc) * (size_t)n];
            }
#pragma unroll
            for (int q = 0; q < kTQ; ++q) {
                const int e = t + q * kBT;
                if (e < kPB * kPB) sh.T[e % kPB][e / kPB] = tq[q];
            }
        }
        __syncthreads();
        for (int rh = wave; rh < nrhs; rh += kBW) {
            gf64 *zp = gb + (size_t)rh * (size_t)n;
            double y = zp[r0 + (lane < bw ? lane : bw - 1)];
            for (int s = bw - 1; s >= 0; --s) {
                const double xs = read_lane(y, s);
                if (lane < s) y = __fma_rn(-sh.T[s][lane], xs, y);  // L^T(lane, s) = L(s, lane)
            }
            if (lane < bw) {
                zp[r0 + lane] = y;
                sh.Ys[rh][lane] = y;
            }
        }
        __syncthreads();
        for (int i = t; i < r0; i += kBT) {
            double l[kPB];  // L(r0 + k, i): column i, contiguous
#pragma unroll
            for (int k = 0; k < kPB; ++k) l[k] = a[(size_t)(r0 + (k < bw ? k : bw - 1)) + (size_t)i * (size_t)n];
            for (int rh = 0; rh < nrhs; ++rh) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < kPB; ++k)
                    if (k < bw) acc = __fma_rn(l[k], sh.Ys[rh][k], acc);
                gf64 *zp = gb + (size_t)rh * (size_t)n;
                zp[i] = zp[i] - acc;
            }
        }
        __syncthreads();
    }
    // grad_B = P^T v: entry perm[i] receives v_i (staged through LDS)
    for (int rh = 0; rh < nrhs; rh += kKC) {
        const int nr = (nrhs - rh) < kKC ? (nrhs - rh) : kKC;
        {
            constexpr int kQ = kKC * kBatchMaxN / kBT;
            double vq[kQ];
            const int tot = nr * n;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = (t + q * kBT) < tot ? (t + q * kBT) : tot - 1;
                vq[q] = gb[(size_t)(rh + e / n) * (size_t)n + e % n];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = t + q * kBT;
                if (e < tot) sh.Lc[e / n][e % n] = vq[q];
            }
        }
        __syncthreads();
        for (int e = t; e < nr * n; e += kBT) {
            const int i = e % n, q = e / n;
            gb[(size_t)(rh + q) * (size_t)n + sh.perm[i]] = sh.Lc[q][i];
        }
        __syncthreads();
    }
    // grad_A = -grad_B X^T: thread per row i, X's rows from LDS, the sum over
    // right-hand sides in order, kKC of them per pass
    for (int rh0 = 0; rh0 < nrhs; rh0 += kKC) {
        const int nr = (nrhs - rh0) < kKC ? (nrhs - rh0) : kKC;
        {
            constexpr int kQ = kKC * kBatchMaxN / kBT;
            double xq[kQ];
            const int tot = nr * n;
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = (t + q * kBT) < tot ? (t + q * kBT) : tot - 1;
                xq[q] = x[(size_t)(rh0 + e / n) * (size_t)n + e % n];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int e = t + q * kBT;
                if (e < tot) sh.Lc[e / n][e % n] = xq[q];
            }
        }
        __syncthreads();
        for (int i = t; i < n; i += kBT) {
            double g[kKC];
#pragma unroll
            for (int q = 0; q < kKC; ++q) g[q] = gb[(size_t)(rh0 + (q < nr ? q : nr - 1)) * (size_t)n + i];
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < kKC; ++q)
                    if (q < nr) s = __fma_rn(g[q], sh.Lc[q][j], s);
                gf64 *gp = ga + (size_t)i + (size_t)j * (size_t)n;
                *gp = (rh0 == 0 ? 0.0 : *gp) - s;
            }
        }
        __syncthreads();
    }
}

// OCC workgroups per CU (systems in flight per CU): 2 * OCC waves per SIMD
template <int OCC>
__global__ __launch_bounds__(kBT, 2 * OCC) void batched_solve_kernel(BatchArgs p)
{
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) sh.job = (int64_t)atomicAdd(p.counter, 1u);
        __syncthreads();
        const int64_t job = sh.job;
        __syncthreads();
        if (job >= p.count) break;  // uniform: every wave leaves together
        const int sys = p.order[job];
        const int n = p.sizes[sys];
        double *a = p.A + p.aoff[sys];
        const int64_t vo = p.voff[sys];
        double *b = p.B + (size_t)vo * (size_t)p.nrhs;
        int32_t *ip = p.ipiv + vo;
        if (p.mode & 1) {
            switch (p.vtab[(n - 1) >> 5]) {  // uniform across the workgroup
            case 0: batch_forward<kVarPB[0], kVarUC[0], OCC>(a, b, ip, n, p.nrhs); break;
            case 1: batch_forward<kVarPB[1], kVarUC[1], OCC>(a, b, ip, n, p.nrhs); break;
            case 2: batch_forward<kVarPB[2], kVarUC[2], OCC>(a, b, ip, n, p.nrhs); break;
            default: batch_forward<kVarPB[3], kVarUC[3], OCC>(a, b, ip, n, p.nrhs); break;
            }
        } else {
            // adjoint only: the row permutation from the stored interchanges
            if (t == 0) {
                sh.info = 0;
                for (int i = 0; i < n; ++i) sh.perm[i] = i;
                for (int k = 0; k < n; ++k) {
                    const int q = ip[k];
                    if (q != k && q >= 0 && q < n) {
                        const int tmp = sh.perm[k];
                        sh.perm[k] = sh.perm[q];
                        sh.perm[q] = tmp;
                    }
                }
            }
            __syncthreads();
        }
        if (p.mode & 2)
            batch_adjoint<OCC>((gcf64 *)a, (gcf64 *)b, (gcf64 *)(p.W + (size_t)vo * (size_t)p.nrhs),
                          (gf64 *)(p.GB + (size_t)vo * (size_t)p.nrhs), (gf64 *)(p.GA + p.aoff[sys]), n, p.nrhs);
        if (t == 0) p.info[sys] = sh.info;
        __syncthreads();
    }
}

}  // namespace

int launch_batched_solve(int64_t count, const int32_t *sizes, const int64_t *aoff, const int64_t *voff,
                         const int32_t *order, double *A, int32_t *ipiv, double *B, const double *W, double *GB,
                         double *GA, int nrhs, int mode, int64_t *info, unsigned *counter, int occ,
                         const signed char *vtab, int cus, hipStream_t st)
{
    if (count <= 0) return HPL_OK;
    if (nrhs < 1 || nrhs > kBatchMaxRhs || mode < 1 || mode > 3 || cus < 1 || (occ != 1 && occ != 2))
        return HPL_ERR_INTERNAL;
    BatchArgs p{count, sizes, aoff, voff, order, A, ipiv, B, W, GB, GA, nrhs, mode, info, counter, {}};
    for (int q = 0; q < kBatchBuckets; ++q) {
        if (vtab[q] < 0 || vtab[q] >= kNumVariants) return HPL_ERR_INTERNAL;
        p.vtab[q] = vtab[q];
    }
    const int64_t wgs = (int64_t)cus * occ;
    const int64_t g = wgs < count ? wgs : count;
    if (occ == 1)
        hipLaunchKernelGGL(batched_solve_kernel<1>, dim3((unsigned)g), dim3(kBT), 0, st, p);
    else
        hipLaunchKernelGGL(batched_solve_kernel<2>, dim3((unsigned)g), dim3(kBT), 0, st, p);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
