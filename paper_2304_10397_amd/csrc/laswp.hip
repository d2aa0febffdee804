// laswp.hip -- applying a panel's row interchanges to other columns (the RS
// phase, Sec. I / Sec. II: all NB pivots found by FACT are applied to the
// rest of the matrix).
//
// The interchanges k = 0..cnt-1 (row r0+k <-> ipiv[k], in order) touch at most
// 2*cnt distinct rows S.  Their composition is a permutation of S, computed
// once per panel by swap_plan_kernel ("slot list": slot s names row rows[s];
// after the interchanges row rows[s] holds the old contents of row
// rows[srcslot[s]]).  Slots 0..cnt-1 are the contiguous rows r0..r0+cnt-1 in
// order, so the reads and writes of that block are coalesced; the other rows
// are scattered (one 8-byte element per column per row: column-major storage
// makes a row interchange a strided access whatever the kernel does).
//
// laswp_kernel then works on a few columns per workgroup: it gathers every
// slot's element into LDS, synchronizes, and writes the permuted values back,
// which is the in-place gather/scatter of the RS phase on one GPU.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kPlanThreads = kMaxSwaps;  // one thread per interchange
constexpr int kHash = 4 * kMaxSwaps;     // open-addressing table of the rows outside the block (load <= 1/4)
constexpr int kHashBits = 11;
static_assert(kHash == 1 << kHashBits, "table size");
constexpr int kLwCols = 8;               // columns per laswp workgroup
constexpr int kLwThreads = 256;

// Workgroup q builds the plan of chunk q: interchanges ipiv[q*kMaxSwaps ...] of
// rows r0 + q*kMaxSwaps ..., output at the given pointers + q*stride.
__global__ __launch_bounds__(kPlanThreads) void swap_plan_kernel(const int32_t *__restrict__ ipiv_all, int64_t total,
                                                                 int64_t r0_all, int64_t nrows, int reverse,
                                                                 int32_t *__restrict__ rows_all,
                                                                 int32_t *__restrict__ src_all,
                                                                 int32_t *__restrict__ nslots_all, int64_t stride,
                                                                 int *__restrict__ err)
{
    const int64_t q = blockIdx.x;
    const int32_t *ipiv = ipiv_all + q * kMaxSwaps;
    const int cnt = (int)((total - q * kMaxSwaps) < kMaxSwaps ? (total - q * kMaxSwaps) : kMaxSwaps);
    const int64_t r0 = r0_all + q * kMaxSwaps;
    int32_t *rows_out = rows_all + q * stride;
    int32_t *src_out = src_all + q * stride;
    int32_t *nslots_out = nslots_all + q * stride;

    __shared__ int piv[kMaxSwaps];        // target row relative to r0 (>= k)
    __shared__ int bslot[kMaxSwaps];      // slot of the target row
    __shared__ int cur[2 * kMaxSwaps];    // content (slot id) currently in slot s
    __shared__ int used[2 * kMaxSwaps];
    __shared__ int pos[2 * kMaxSwaps];    // compacted position of slot s
    __shared__ int scan[kPlanThreads];
    __shared__ int hkey[kHash];           // outside row (relative to r0), or -1
    __shared__ int hfirst[kHash];         // its first interchange index
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int e = t; e < kHash; e += kPlanThreads) {
        hkey[e] = -1;
        hfirst[e] = kMaxSwaps;
    }
    __syncthreads();
    if (t < cnt) {
        const int64_t p = ipiv[t];
        // an interchange partner must lie in [r0 + k, nrows): anything else would
        // address rows outside the matrix, so the plan is dropped and reported
        if (p < r0 + t || p >= nrows) atomicOr(&bad, 1);
        piv[t] = (int)(p - r0);
    }
    __syncthreads();
    if (bad) {
        if (t == 0) {
            *nslots_out = 0;
            atomicOr(err, 1);
        }
        return;
    }
    // a row outside the contiguous block takes slot cnt + (its first interchange
    // index): the rows are entered into an LDS hash table (linear probing; at
    // most cnt keys in 4 cnt entries, so every probe sequence ends), which
    // keeps the smallest interchange index of each row
    int hs = -1;
    if (t < cnt && piv[t] >= cnt) {
        const int p = piv[t];
        int hh = (int)(((unsigned)p * 2654435761u) >> (32 - kHashBits));
        for (int probe = 0; probe < kHash; ++probe) {
            const int old = atomicCAS(&hkey[hh], -1, p);
            if (old == -1 || old == p) {
                hs = hh;
                break;
            }
            hh = (hh + 1) & (kHash - 1);
        }
        if (hs >= 0) atomicMin(&hfirst[hs], t);
    }
    __syncthreads();
    if (t < cnt) {
        const int p = piv[t];
        bslot[t] = (p >= cnt) ? cnt + (hs >= 0 ? hfirst[hs] : t) : p;
    }
    __syncthreads();
    for (int s = t; s < 2 * cnt; s += kPlanThreads)
        used[s] = (s < cnt) ? 1 : (bslot[s - cnt] == s ? 1 : 0);
    // cur[s] = the slot whose content ends in slot s once the interchanges
    // (k, bslot[k]) are applied in order: followed back from s through them,
    // last applied first -- independent per slot, so every thread takes its own
    for (int s = t; s < 2 * cnt; s += kPlanThreads) {
        int p = s;
        for (int kk = cnt - 1; kk >= 0; --kk) {
            const int k = reverse ? cnt - 1 - kk : kk;
            const int b = bslot[k];
            p = (p == k) ? b : (p == b ? k : p);
        }
        cur[s] = p;
    }
    __syncthreads();
    // exclusive scan of used[] over 2*cnt slots: thread t owns slots 2t, 2t+1
    const int s0 = 2 * t, s1 = 2 * t + 1;
    const int u0 = (s0 < 2 * cnt) ? used[s0] : 0, u1 = (s1 < 2 * cnt) ? used[s1] : 0;
    scan[t] = u0 + u1;
    __syncthreads();
    for (int o = 1; o < kPlanThreads; o <<= 1) {
        const int v = (t >= o) ? scan[t - o] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    const int base = scan[t] - (u0 + u1);
    if (s0 < 2 * cnt) pos[s0] = base;
    if (s1 < 2 * cnt) pos[s1] = base + u0;
    __syncthreads();
    for (int s = t; s < 2 * cnt; s += kPlanThreads) {
        if (!used[s]) continue;
        const int rel = (s < cnt) ? s : piv[s - cnt];
        rows_out[pos[s]] = (int32_t)(r0 + rel);
        src_out[pos[s]] = pos[cur[s]];
    }
    if (t == kPlanThreads - 1) *nslots_out = scan[t];
}

__global__ __launch_bounds__(kLwThreads) void laswp_kernel(double *__restrict__ A, int64_t lda, int64_t col0,
                                                           int64_t ncols, const int32_t *__restrict__ rows,
                                                           const int32_t *__restrict__ srcslot,
                                                           const int32_t *__restrict__ nslots_p)
{
    // column groups of kLwCols, taken grid-stride (the grid may be smaller than
    // the number of groups, so that the interchange leaves CUs to other work)
    __shared__ double vals[2 * kMaxSwaps][kLwCols];
    const int ns = *nslots_p;
    const int64_t ngroups = (ncols + kLwCols - 1) / kLwCols;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t cb = col0 + grp * kLwCols;
        const int64_t left = col0 + ncols - cb;
        const int nc = left < kLwCols ? (int)left : kLwCols;
        for (int s = threadIdx.x; s < ns; s += kLwThreads) {
            const int64_t r = rows[s];
#pragma unroll
            for (int c = 0; c < kLwCols; ++c)  // entries past nc are never written back
                vals[s][c] = load_or(c < nc, A + off(r, cb + c, lda), A + off(r, cb, lda), 0.0);
        }
        __syncthreads();
        for (int s = threadIdx.x; s < ns; s += kLwThreads) {
            const int ss = srcslot[s];
            if (ss == s) continue;
            const int64_t r = rows[s];
#pragma unroll
            for (int c = 0; c < kLwCols; ++c)
                if (c < nc) A[off(r, cb + c, lda)] = vals[ss][c];
        }
        __syncthreads();  // vals is refilled by the next group
    }
}

}  // namespace

int launch_swap_plan(const int32_t *ipiv, int cnt, int64_t r0, int64_t nrows, bool reverse, SwapPlan plan,
                     hipStream_t st)
{
    if (cnt <= 0 || cnt > kMaxSwaps) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(swap_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, ipiv, (int64_t)cnt, r0, nrows,
                       reverse ? 1 : 0, plan.rows, plan.srcslot, plan.nslots, (int64_t)0, plan.err);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_swap_plans_all(const int32_t *ipiv, int64_t total, int64_t r0, int64_t nrows, bool reverse,
                          int32_t *plans, int *err, hipStream_t st)
{
    if (total <= 0) return HPL_OK;
    const int64_t nchunks = (total + kMaxSwaps - 1) / kMaxSwaps;
    if (nchunks > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(swap_plan_kernel, dim3((unsigned)nchunks), dim3(kPlanThreads), 0, st, ipiv, total, r0, nrows,
                       reverse ? 1 : 0, plans, plans + 2 * kMaxSwaps, plans + 4 * kMaxSwaps, (int64_t)kPlanStride,
                       err);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int launch_laswp(double *A, int64_t lda, int64_t col0, int64_t ncols, SwapPlan plan, int64_t max_wgs,
                 hipStream_t st)
{
    if (ncols <= 0) return HPL_OK;
    int64_t g = (ncols + kLwCols - 1) / kLwCols;
    if (max_wgs > 0 && g > max_wgs) g = max_wgs;
    if (g > 0x7fffffffll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)g), dim3(kLwThreads), 0, st, A, lda, col0, ncols, plan.rows,
                       plan.srcslot, plan.nslots);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
