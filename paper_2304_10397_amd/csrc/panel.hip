// panel.hip -- leaf of the recursive panel factorization (FACT).
//
// FACT LU-factors the tall, skinny slab of the current columns with
// interchanges restricted to those columns (Sec. II).  The paper runs it on the
// CPU, splitting the slab into row tiles owned by threads, with the pivot
// search a reduction over threads and the tile holding the diagonal on the
// main thread (Sec. III-A).  Here the same decomposition is mapped onto the
// GPU: G workgroups each own a contiguous range of the slab's rows (workgroup
// 0 owns the first rows, which hold the diagonal and receive the pivot rows),
// and each column costs one grid-wide barrier:
//
//   1. every workgroup reduces its rows to a candidate (|a|, row) with wave
//      shuffles and LDS, and publishes it with a copy of that row's w values
//      (workgroup 0 also publishes the current diagonal row);
//   2. barrier (monotonic atomic counter, agent-scope release/acquire);
//   3. every workgroup reduces the G candidates identically (largest |a|, the
//      lowest row on ties -- independent of the reduction order), so all
//      agree on the pivot row p and read its values without touching it;
//   4. workgroup 0 writes the pivot row into the diagonal row, the owner of p
//      writes the old diagonal row into row p, and every workgroup divides its
//      rows by the pivot (true division) and applies the rank-1 update to the
//      remaining leaf columns, tracking the next column's candidate on the way.
//
// Candidate slots are double-buffered by column parity, so a workgroup that
// races ahead to column k+1 never overwrites what a slower one still reads for
// column k.  Every wait is bounded (wall clock); on time-out the kernel raises
// a flag, all workgroups leave, and the host reports HPL_ERR_INTERNAL.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kLeafThreads = 256;
constexpr int kLeafWaves = kLeafThreads / 64;
constexpr unsigned long long kSpinLimit = 3000000000ull;  // 30 s of the 100 MHz wall clock

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi)
{
    return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void wave_argmax(double &v, int64_t &i)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int64_t oi = __shfl_xor(i, o, 64);
        if (better(ov, oi, v, i)) { v = ov; i = oi; }
    }
}

__device__ __forceinline__ double ld_agent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kLeafThreads) void panel_leaf_kernel(double *__restrict__ A, int64_t lda, int64_t c,
                                                                  int64_t m, int w, int32_t *__restrict__ ipiv,
                                                                  LeafSync sync, unsigned long long bar_base,
                                                                  int G, int64_t R)
{
    __shared__ double u[kLeafMaxW];
    __shared__ double tr[kLeafMaxW];
    __shared__ double rv[kLeafWaves];
    __shared__ int64_t ri[kLeafWaves];
    __shared__ double s_pv;
    __shared__ int64_t s_p;
    __shared__ int s_gw;
    __shared__ int s_abort;

    double *S = A + off(c, c, lda);  // slab(i, j) = S[i + j*lda], 0 <= i < m, 0 <= j < w
    const int g = blockIdx.x, t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int64_t rbeg = (int64_t)g * R;
    const int64_t rend = (rbeg + R) < m ? (rbeg + R) : m;

    double bv = -1.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = rbeg + t; i < rend; i += kLeafThreads) {
        const double v = fabs(S[i]);
        if (better(v, i, bv, bi)) { bv = v; bi = i; }
    }

    for (int k = 0; k < w; ++k) {
        const int par = k & 1;
        // ---- 1. local candidate
        wave_argmax(bv, bi);
        if (lane == 0) { rv[wid] = bv; ri[wid] = bi; }
        __syncthreads();
        if (t == 0) {
            double v = rv[0];
            int64_t i = ri[0];
            for (int q = 1; q < kLeafWaves; ++q)
                if (better(rv[q], ri[q], v, i)) { v = rv[q]; i = ri[q]; }
            s_pv = v;
            s_p = i;
        }
        __syncthreads();
        double *slot = sync.slots + ((size_t)par * kLeafMaxWGs + g) * kLeafSlot;
        const int64_t cand = s_p;
        if (t == 0) {
            slot[0] = s_pv;
            slot[1] = __longlong_as_double(cand);
        }
        if (t < w && cand != INT64_MAX) slot[2 + t] = S[cand + (int64_t)t * lda];
        if (g == 0 && t < w) sync.top[par * kLeafMaxW + t] = S[k + (int64_t)t * lda];
        // ---- 2. grid barrier
        __syncthreads();
        if (t == 0) {
            int ab = 0;
            if (G > 1) {
                __threadfence();
                atomicAdd(sync.counter, 1ull);
                const unsigned long long target = bar_base + (unsigned long long)G * (unsigned long long)(k + 1);
                const unsigned long long t0 = wall_clock64();
                while (__hip_atomic_load(sync.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    if (__hip_atomic_load(sync.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ab = 1; break; }
                    if (wall_clock64() - t0 > kSpinLimit) {
                        __hip_atomic_store(sync.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ab = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __threadfence();
            }
            s_abort = ab;
        }
        __syncthreads();
        if (s_abort) return;
        // ---- 3. global pivot: every workgroup reduces all candidates the same way
        double gv = -1.0;
        int64_t gi = INT64_MAX;
        for (int q = t; q < G; q += kLeafThreads) {
            const double *sq = sync.slots + ((size_t)par * kLeafMaxWGs + q) * kLeafSlot;
            const double v = ld_agent(sq);
            const int64_t i = __double_as_longlong(ld_agent(sq + 1));
            if (better(v, i, gv, gi)) { gv = v; gi = i; }
        }
        wave_argmax(gv, gi);
        if (lane == 0) { rv[wid] = gv; ri[wid] = gi; }
        __syncthreads();
        if (t == 0) {
            double v = rv[0];
            int64_t i = ri[0];
            for (int q = 1; q < kLeafWaves; ++q)
                if (better(rv[q], ri[q], v, i)) { v = rv[q]; i = ri[q]; }
            s_pv = v;
            s_p = i;
            const int64_t owner = (i == INT64_MAX) ? 0 : i / R;  // the owner of the pivot row published it
            s_gw = (int)(owner < G ? owner : G - 1);
        }
        __syncthreads();
        const double pv = s_pv;
        const int64_t p = s_p;
        const bool singular = !(pv > 0.0);
        if (t < w) {
            const double *sw = sync.slots + ((size_t)par * kLeafMaxWGs + s_gw) * kLeafSlot;
            u[t] = singular ? 0.0 : ld_agent(sw + 2 + t);
            tr[t] = ld_agent(sync.top + par * kLeafMaxW + t);
        }
        if (g == 0 && t == 0) {
            ipiv[c + k] = (int32_t)(c + (singular ? k : p));
            if (singular) atomicMin(sync.info, (unsigned long long)(c + k + 1));
        }
        __syncthreads();
        // ---- 4. interchange, scale, rank-1 update; next column's candidate
        const int64_t pp = singular ? (int64_t)k : p;
        if (pp != k) {
            if (g == 0 && t < w) S[k + (int64_t)t * lda] = u[t];
            if (pp >= rbeg && pp < rend && t < k) S[pp + (int64_t)t * lda] = tr[t];
        }
        bv = -1.0;
        bi = INT64_MAX;
        const bool next = (k + 1 < w);
        const int64_t istart = (rbeg > k + 1 ? rbeg : (int64_t)k + 1) + t;
        if (singular) {
            if (next)
                for (int64_t i = istart; i < rend; i += kLeafThreads) {
                    const double v = fabs(S[i + (int64_t)(k + 1) * lda]);
                    if (better(v, i, bv, bi)) { bv = v; bi = i; }
                }
        } else {
            const double piv = u[k];
            for (int64_t i = istart; i < rend; i += kLeafThreads) {
                double *row = S + i;
                const bool swapped = (i == pp);
                const double l = (swapped ? tr[k] : row[(int64_t)k * lda]) / piv;
                row[(int64_t)k * lda] = l;
                for (int j = k + 1; j < w; ++j) {
                    const double a = swapped ? tr[j] : row[(int64_t)j * lda];
                    const double nv = a - l * u[j];
                    row[(int64_t)j * lda] = nv;
                    if (j == k + 1) {
                        const double v = fabs(nv);
                        if (better(v, i, bv, bi)) { bv = v; bi = i; }
                    }
                }
            }
        }
    }
}

}  // namespace

int leaf_groups(int64_t m, int w, int gmax)
{
    const int64_t rmin = 256;
    int64_t g = (m + rmin - 1) / rmin;
    if (g > gmax) g = gmax;
    if (g < 1) g = 1;
    // workgroup 0 must own the first w rows
    while (g > 1 && (m + g - 1) / g < w) --g;
    return (int)g;
}

int launch_panel_leaf(double *A, int64_t lda, int64_t c, int64_t m, int w, int32_t *ipiv, LeafSync sync,
                      unsigned long long bar_base, int G, hipStream_t st)
{
    if (w <= 0 || w > kLeafMaxW || G < 1 || G > kLeafMaxWGs || m < w) return HPL_ERR_INTERNAL;
    const int64_t R = (m + G - 1) / G;
    hipLaunchKernelGGL(panel_leaf_kernel, dim3(G), dim3(kLeafThreads), 0, st, A, lda, c, m, w, ipiv, sync,
                       bar_base, G, R);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

}  // namespace hplx
