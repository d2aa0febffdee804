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
                    const double nv = __fma_rn(-l, u[j], a);
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

// ---------------------------------------------------------------------------
// Register-resident leaf.  Thread t of workgroup g holds rows rbeg + t + 512q
// (q < 2) of the leaf in registers; v[q][j] is the row's value in column k + j
// at step k (the active columns rotate down by one each step, so every register
// index is a compile-time constant).  Column k of every active row is written
// to memory at step k; the U row is written by workgroup 0.
//
// Cross-workgroup exchange without fences or counters: every published 64-bit
// word carries a 32-bit tag (unique per launch and step) and 32 bits of
// payload; writers use relaxed agent-scope atomic stores, readers poll with
// relaxed agent-scope atomic loads until each word they need shows the current
// tag, so each word validates itself and no ordering between words is needed.
// Each step costs two short round trips: every workgroup reads the G
// candidates' keys (one word per thread, polled side by side), picks the pivot
// locally, then reads only the winner's row and the diagonal row (both halves
// of each value loaded together).
// Slot of workgroup g: words 0..2 = tagged (row index, |a| low, |a| high),
// words 3 + 2j, 4 + 2j = tagged halves of the candidate row's value in column
// k + j.  The diagonal row is published by workgroup 0 in a separate area.
//
// The interchanges of the leaf's own finished L columns (columns < k at step
// k) are not done here; leaf_left_swaps_kernel applies them afterwards.
// ---------------------------------------------------------------------------
constexpr int kRegW = 32;                        // leaf width handled in registers
constexpr int kRegRPT = 2;                       // rows per thread
constexpr int kRegThreads = 512;
constexpr int kRegWaves = kRegThreads / 64;
constexpr int kRegRows = kRegThreads * kRegRPT;  // rows per workgroup (max)

__device__ __forceinline__ void put_tagged(unsigned long long *p, uint32_t tag, uint32_t payload)
{
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spins until *p carries tag (or the abort flag rises / the wall-clock limit
// passes).  The abort flag and the clock are looked at only every 32nd poll:
// each look is another trip to memory, and a poll loop that made it every time
// would see the awaited word up to one such trip late.
__device__ __forceinline__ bool get_tagged(const unsigned long long *p, uint32_t tag, uint32_t &payload,
                                           int *abort_flag, unsigned long long t0)
{
    for (unsigned it = 1;; ++it) {
        const unsigned long long v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == tag) {
            payload = (uint32_t)v;
            return true;
        }
        if ((it & 31u) == 0) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
            if (wall_clock64() - t0 > kSpinLimit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// The two words of one value: both loads are issued before either is tested,
// so a pair that is already there costs one round trip rather than two; a word
// that does not carry the tag yet is then polled on its own.  A word loaded
// early with the current tag holds the current payload (tags are unique per
// launch and step), so using it is as safe as polling it again.
__device__ __forceinline__ bool get_tagged_pair(const unsigned long long *p, uint32_t tag, uint32_t &lo,
                                                uint32_t &hi, int *abort_flag, unsigned long long t0)
{
    const unsigned long long v0 = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long v1 = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(v0 >> 32) == tag)
        lo = (uint32_t)v0;
    else if (!get_tagged(p, tag, lo, abort_flag, t0))
        return false;
    if ((uint32_t)(v1 >> 32) == tag)
        hi = (uint32_t)v1;
    else if (!get_tagged(p + 1, tag, hi, abort_flag, t0))
        return false;
    return true;
}

__device__ __forceinline__ double dbl_of(uint32_t lo, uint32_t hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Largest v over the workgroup, the lowest row i among its holders on ties
// (every v >= -1, rows below 2^31 or INT64_MAX for none).  The wave's maximum
// and the lowest row holding it go through DPP and lane reads; the eight wave
// results meet in rv/ri behind one barrier.  rv/ri are read after that barrier
// and written again only on the next call: a caller must pass a barrier of its
// own between two calls with the same arrays.
__device__ __forceinline__ void block_argmax512(double &v, int64_t &i, double *rv, unsigned *ri)
{
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const double m = wave_max(v);
    const unsigned r = wave_min_u32(v == m ? (unsigned)i : 0xffffffffu);
    if (lane == 0) { rv[wid] = m; ri[wid] = r; }
    __syncthreads();
    double bv = rv[0];
    unsigned br = ri[0];
#pragma unroll
    for (int q = 1; q < kRegWaves; ++q) {
        const double x = rv[q];
        const unsigned y = ri[q];
        if (x > bv || (x == bv && y < br)) { bv = x; br = y; }
    }
    v = bv;
    i = (br == 0xffffffffu) ? INT64_MAX : (int64_t)br;
}

__global__ __launch_bounds__(kRegThreads) void leaf_reg_kernel(double *__restrict__ A, int64_t lda, int64_t c,
                                                               int64_t m, int w, int32_t *__restrict__ ipiv,
                                                               LeafSync sync, uint32_t tag0, int G, int64_t R)
{
    __shared__ double cand[kRegW];   // candidate row (active columns) of this workgroup
    __shared__ double topv[kRegW];   // diagonal row (workgroup 0)
    __shared__ double u[kRegW];      // pivot row, active columns
    __shared__ double tr[kRegW];     // old diagonal row, active columns
    __shared__ double rv[kRegWaves];
    __shared__ unsigned ri[kRegWaves];
    __shared__ int s_abort;
    __shared__ uint32_t xw[3 * kLeafMaxWGs + 4 * kRegW];  // payloads of one exchange: keys, then two rows

    double *S = A + off(c, c, lda);
    const int g = blockIdx.x, t = threadIdx.x;
    const int64_t rbeg = (int64_t)g * R;
    const int64_t rend = (rbeg + R) < m ? (rbeg + R) : m;
    unsigned long long *slots = sync.tslots;
    unsigned long long *topw = sync.ttop;
    const unsigned long long t0 = wall_clock64();

    double v[kRegRPT][kRegW];
    int64_t row[kRegRPT];
    double bv = -1.0;
    int64_t bi = INT64_MAX;
#pragma unroll
    for (int q = 0; q < kRegRPT; ++q) {
        row[q] = rbeg + t + (int64_t)q * kRegThreads;
        const bool live = row[q] < rend;
#pragma unroll
        for (int j = 0; j < kRegW; ++j) v[q][j] = (live && j < w) ? S[off(row[q], j, lda)] : 0.0;
        if (live) {
            const double a = fabs(v[q][0]);
            if (better(a, row[q], bv, bi)) { bv = a; bi = row[q]; }
        }
    }
    if (t == 0) s_abort = 0;

    // Register slots at and beyond the active count hold values that are never
    // used; the copies and the rank-1 update run over all kRegW slots without
    // per-slot tests (a test per slot costs a branch per slot and step).
    for (int k = 0; k < w; ++k) {
        const int na = w - k;  // active columns
        const uint32_t tag = tag0 + (uint32_t)k + 1u;
        const int par = k & 1;
        // ---- 1. this workgroup's candidate (one barrier)
        block_argmax512(bv, bi, rv, ri);
        double pv;
        int64_t p;
        bool singular;
        if (G == 1) {
#pragma unroll
            for (int q = 0; q < kRegRPT; ++q) {
                if (row[q] == bi && row[q] < rend) {
#pragma unroll
                    for (int j = 0; j < kRegW; ++j) cand[j] = v[q][j];
                }
                if (row[q] == k) {
#pragma unroll
                    for (int j = 0; j < kRegW; ++j) topv[j] = v[q][j];
                }
            }
            __syncthreads();
            pv = bv;
            p = bi;
            singular = !(pv > 0.0);
            if (t < na) {
                tr[t] = topv[t];
                u[t] = singular ? topv[t] : cand[t];  // singular: no interchange, u is the diagonal row
            }
        } else {
            // ---- 2. publish (tagged words, no fences): the key, then the
            //      candidate row and (workgroup 0) the diagonal row, each sent
            //      by the wave that holds it: the holding lane puts the row in
            //      LDS and its wave reads it back one value per lane (the LDS
            //      operations of one wave complete in order).  A workgroup
            //      without a candidate still sends tagged words, so that no
            //      reader ever waits on a slot that is not written.
            unsigned long long *my = slots + ((size_t)par * kLeafMaxWGs + g) * kLeafSlotWords;
            if (t == 0) put_tagged(my, tag, (uint32_t)bi);
            if (t == 1) put_tagged(my + 1, tag, (uint32_t)(__double_as_longlong(bv)));
            if (t == 2) put_tagged(my + 2, tag, (uint32_t)((unsigned long long)__double_as_longlong(bv) >> 32));
            const int lane = t & 63;
            const bool mine = bi != INT64_MAX && (row[0] == bi || row[1] == bi);
            if (__ballot(mine) != 0) {
                if (mine) {
                    const bool q0 = row[0] == bi;
#pragma unroll
                    for (int j = 0; j < kRegW; ++j) cand[j] = q0 ? v[0][j] : v[1][j];
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (lane < 2 * na) {
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(cand[lane >> 1]);
                    put_tagged(my + 3 + lane, tag, (lane & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits);
                }
            } else if (bi == INT64_MAX && t < 2 * na) {
                put_tagged(my + 3 + t, tag, 0u);
            }
            if (g == 0) {
                const bool diag = row[0] == k || row[1] == k;
                if (__ballot(diag) != 0) {
                    if (diag) {
                        const bool q0 = row[0] == k;
#pragma unroll
                        for (int j = 0; j < kRegW; ++j) topv[j] = q0 ? v[0][j] : v[1][j];
                    }
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    if (lane < 2 * na) {
                        const unsigned long long bits = (unsigned long long)__double_as_longlong(topv[lane >> 1]);
                        put_tagged(topw + (size_t)par * 2 * kRegW + lane, tag,
                                   (lane & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits);
                    }
                }
            }
            // ---- 3. two short round trips.  (a) every candidate's key (row,
            //      |a|): one tagged word per thread, so the polls of a step run
            //      side by side rather than one after another
            for (int e = t; e < 3 * G; e += kRegThreads) {
                uint32_t pay = 0;
                const int q = e / 3, wi = e - 3 * q;
                const unsigned long long *src = slots + ((size_t)par * kLeafMaxWGs + q) * kLeafSlotWords + wi;
                if (!get_tagged(src, tag, pay, sync.abort_flag, t0)) s_abort = 1;
                xw[e] = pay;
            }
            __syncthreads();
            if (s_abort) return;
            // every wave reduces the G keys itself (largest |a|, lowest row on
            // ties), so that no further barrier is needed
            {
                double gv = -1.0;
                unsigned gr = 0xffffffffu;
                for (int e = lane; e < G; e += 64) {
                    const double x = dbl_of(xw[3 * e + 1], xw[3 * e + 2]);
                    const unsigned y = xw[3 * e];
                    if (x > gv || (x == gv && y < gr)) { gv = x; gr = y; }
                }
                pv = wave_max(gv);
                const unsigned r = wave_min_u32(gv == pv ? gr : 0xffffffffu);
                p = (r == 0xffffffffu) ? INT64_MAX : (int64_t)r;
            }
            singular = !(pv > 0.0);
            // (b) the winner's row and the diagonal row: each thread t < 2 na
            //     takes one value (its two tagged halves)
            const int64_t owner0 = (p == INT64_MAX) ? 0 : p / R;
            const int owner = (int)(owner0 < G ? owner0 : G - 1);
            if (t < 2 * na) {
                const bool top = t >= na;
                const int j = top ? t - na : t;
                const unsigned long long *src =
                    top ? topw + (size_t)par * 2 * kRegW + 2 * j
                        : slots + ((size_t)par * kLeafMaxWGs + owner) * kLeafSlotWords + 3 + 2 * j;
                uint32_t lo = 0, hi = 0;
                if (!get_tagged_pair(src, tag, lo, hi, sync.abort_flag, t0)) s_abort = 1;
                const double x = dbl_of(lo, hi);
                if (top) {
                    tr[j] = x;
                    if (singular) u[j] = x;  // no interchange: u is the diagonal row
                } else if (!singular) {
                    u[j] = x;
                }
            }
        }
        __syncthreads();
        if (s_abort) return;
        if (singular) p = k;
        if (g == 0 && t == 0) {
            ipiv[c + k] = (int32_t)(c + p);
            if (singular) atomicMin(sync.info, (unsigned long long)(c + k + 1));
        }
        // ---- 5. U row k, interchange of the active parts, scale, rank-1 update
        if (g == 0 && t < na) S[off(k, k + t, lda)] = u[t];
        double uu[kRegW];
#pragma unroll
        for (int j = 0; j < kRegW; ++j) uu[j] = u[j];
        const double piv = uu[0];
        bv = -1.0;
        bi = INT64_MAX;
#pragma unroll
        for (int q = 0; q < kRegRPT; ++q) {
            const int64_t i = row[q];
            if (i >= rend || i <= k) continue;
            if (i == p) {
#pragma unroll
                for (int j = 0; j < kRegW; ++j) v[q][j] = tr[j];
            }
            const double l = singular ? v[q][0] : v[q][0] / piv;
            S[off(i, k, lda)] = l;
            if (singular) {
#pragma unroll
                for (int j = 1; j < kRegW; ++j) v[q][j - 1] = v[q][j];
            } else {
#pragma unroll
                for (int j = 1; j < kRegW; ++j) v[q][j - 1] = __fma_rn(-l, uu[j], v[q][j]);
            }
            if (na > 1) {
                const double a = fabs(v[q][0]);
                if (better(a, i, bv, bi)) { bv = a; bi = i; }
            }
        }
    }
}

// In-leaf interchanges of the finished L columns: column c + j receives the
// interchanges k = j+1 .. w-1 of the leaf (rows c+k <-> ipiv[c+k]), composed
// into a permutation of the touched rows and applied by gather/scatter.
__global__ __launch_bounds__(64) void leaf_left_swaps_kernel(double *__restrict__ A, int64_t lda, int64_t c, int w,
                                                             const int32_t *__restrict__ ipiv)
{
    __shared__ int64_t rows[2 * kRegW];
    __shared__ int cont[2 * kRegW];
    __shared__ double vals[2 * kRegW];
    __shared__ int64_t piv[kRegW];
    __shared__ int bslot[kRegW];
    __shared__ int ns;
    const int j = blockIdx.x, t = threadIdx.x;
    const int cnt = w - 1 - j;  // interchanges k = j+1 .. w-1
    if (t < w) piv[t] = ipiv[c + t];
    __syncthreads();
    // slots: 0..cnt-1 are rows c+j+1 .. c+w-1; an outside row p gets slot cnt + (f - j - 1)
    // where f is its first interchange index after j (found in parallel, one k per lane)
    if (t > j && t < w) {
        const int64_t p = piv[t];
        int b;
        if (p < c + w) {
            b = (int)(p - (c + j + 1));
        } else {
            int f = t;
            for (int k2 = j + 1; k2 < t; ++k2)
                if (piv[k2] == p) { f = k2; break; }
            b = cnt + (f - j - 1);
            if (f == t) rows[b] = p;
        }
        bslot[t] = b;
    }
    if (t < cnt) rows[t] = c + j + 1 + t;
    if (t < 2 * cnt) cont[t] = t;
    __syncthreads();
    if (t == 0) {
        for (int k = j + 1; k < w; ++k) {
            const int a = k - j - 1, b = bslot[k];
            const int ca = cont[a];
            cont[a] = cont[b];
            cont[b] = ca;
        }
        ns = 2 * cnt;
    }
    __syncthreads();
    // slot cnt + q is in use only if some interchange put an outside row there
    double *col = A + off(0, c + j, lda);
    const bool used = (t < cnt) || (t >= cnt && t < 2 * cnt && bslot[t - cnt + j + 1] == t);
    if (t < ns && used) vals[t] = col[rows[t]];
    __syncthreads();
    if (t < ns && used && cont[t] != t) col[rows[t]] = vals[cont[t]];
}

}  // namespace

int leaf_reg_groups(int64_t m, int w)
{
    if (w > kRegW) return 0;
    const int64_t g = (m + kRegRows - 1) / kRegRows;
    return g <= kLeafMaxWGs ? (int)g : 0;
}

int launch_leaf_reg(double *A, int64_t lda, int64_t c, int64_t m, int w, int32_t *ipiv, LeafSync sync, uint32_t tag0,
                    int G, hipStream_t st)
{
    if (w <= 0 || w > kRegW || G < 1 || G > kLeafMaxWGs || m < w) return HPL_ERR_INTERNAL;
    const int64_t R = (m + G - 1) / G;
    if (R > kRegRows || R < w) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(leaf_reg_kernel, dim3(G), dim3(kRegThreads), 0, st, A, lda, c, m, w, ipiv, sync, tag0, G, R);
    HPLX_TRY_LAUNCH();
    if (w > 1) {
        hipLaunchKernelGGL(leaf_left_swaps_kernel, dim3(w - 1), dim3(64), 0, st, A, lda, c, w, (const int32_t *)ipiv);
        HPLX_TRY_LAUNCH();
    }
    return HPL_OK;
}

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
