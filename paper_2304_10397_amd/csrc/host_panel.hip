// host_panel.hip -- the paper's CPU FACT (Sec. III-A, the multi-threaded panel
// factorization, and its Fig. of tiles dealt round-robin to T threads), kept as
// a comparison variant of the GPU panel.
//
// The m x nb panel (host memory, column-major) is split into tiles of nb rows;
// tile i belongs to thread i mod T, so thread 0 owns the tile holding the
// diagonal block.  The factorization is recursive right-looking with two
// halves per level down to a base of 16 columns, right-looking inside the base:
//   * pivot of column k: every thread finds the largest |a_ik| over its rows
//     i >= k (ties: the lowest row), thread 0 reduces the T candidates,
//     interchanges the two rows across all nb columns of the panel and records
//     the pivot;
//   * every thread then divides its rows below k by the pivot and applies the
//     rank-1 update to the base block's remaining columns;
//   * between the halves of a level thread 0 solves U12 = L11^{-1} A12 and every
//     thread updates its rows of A22 -= L21 U12.
// Threads meet at a spin barrier (two per column).  Host code only: nothing
// here runs on the GPU.
#include "common.hpp"

#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

namespace hplx {

namespace {

constexpr int64_t kHostBase = 16;

class SpinBarrier {
public:
    explicit SpinBarrier(int n) : n_(n) {}
    void wait()
    {
        const int gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            gen_.fetch_add(1, std::memory_order_acq_rel);
        } else {
            int spins = 0;
            while (gen_.load(std::memory_order_acquire) == gen)
                if (++spins > 4096) {
                    std::this_thread::yield();
                    spins = 0;
                }
        }
    }

private:
    const int n_;
    std::atomic<int> count_{0};
    std::atomic<int> gen_{0};
};

struct HostPanel {
    double *P;
    int64_t m, nb, ld;
    int32_t *ipiv;
    int T;
    SpinBarrier bar;
    std::vector<double> cval;
    std::vector<int64_t> crow;
    double piv = 0.0;
    int64_t info = 0;
    HostPanel(double *P_, int64_t m_, int64_t nb_, int64_t ld_, int32_t *ip_, int T_)
        : P(P_), m(m_), nb(nb_), ld(ld_), ipiv(ip_), T(T_), bar(T_), cval(T_), crow(T_)
    {
    }
    double &at(int64_t i, int64_t j) { return P[i + j * ld]; }

    // row ranges [r0, r1) within [lo, m) owned by thread tid, tile by tile
    template <typename F> void own_ranges(int tid, int64_t lo, F &&f)
    {
        const int64_t ntiles = (m + nb - 1) / nb;
        for (int64_t tile = tid; tile < ntiles; tile += T) {
            int64_t r0 = tile * nb, r1 = r0 + nb < m ? r0 + nb : m;
            if (r0 < lo) r0 = lo;
            if (r0 < r1) f(r0, r1);
        }
    }

    void base(int tid, int64_t c, int64_t w)
    {
        for (int64_t k = c; k < c + w; ++k) {
            double best = -1.0;
            int64_t brow = -1;
            own_ranges(tid, k, [&](int64_t r0, int64_t r1) {
                const double *col = &at(0, k);
                for (int64_t i = r0; i < r1; ++i) {
                    const double v = std::fabs(col[i]);
                    if (v > best) {  // rows visited in increasing order: the first maximum is the lowest row
                        best = v;
                        brow = i;
                    }
                }
            });
            cval[tid] = best;
            crow[tid] = brow;
            bar.wait();
            if (tid == 0) {
                double gv = -1.0;
                int64_t p = -1;
                for (int q = 0; q < T; ++q)
                    if (crow[q] >= 0 && (cval[q] > gv || (cval[q] == gv && crow[q] < p))) {
                        gv = cval[q];
                        p = crow[q];
                    }
                if (p < 0) p = k;  // a NaN column: keep the diagonal row
                ipiv[k] = (int32_t)p;
                if (p != k)
                    for (int64_t j = 0; j < nb; ++j) {
                        const double x = at(k, j);
                        at(k, j) = at(p, j);
                        at(p, j) = x;
                    }
                piv = at(k, k);
                if (piv == 0.0 && info == 0) info = k + 1;  // column left unscaled
            }
            bar.wait();
            const double pv = piv;
            if (pv != 0.0) {
                // l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj column by column
                own_ranges(tid, k + 1, [&](int64_t r0, int64_t r1) {
                    double *lk = &at(0, k);
                    for (int64_t i = r0; i < r1; ++i) lk[i] = lk[i] / pv;
                    for (int64_t j = k + 1; j < c + w; ++j) {
                        const double u = at(k, j);
                        double *cj = &at(0, j);
                        for (int64_t i = r0; i < r1; ++i) cj[i] = cj[i] - lk[i] * u;
                    }
                });
            }
        }
        bar.wait();
    }

    void rec(int tid, int64_t c, int64_t w)
    {
        if (w <= kHostBase) {
            base(tid, c, w);
            return;
        }
        int64_t w1 = (w / 2 + kHostBase - 1) / kHostBase * kHostBase;
        if (w1 >= w) w1 = w / 2;
        const int64_t w2 = w - w1;
        rec(tid, c, w1);
        // U12 = L11^{-1} A12 (unit lower, forward substitution, thread 0)
        if (tid == 0)
            for (int64_t j = c + w1; j < c + w; ++j)
                for (int64_t i = c; i < c + w1; ++i) {
                    double s = at(i, j);
                    for (int64_t k = c; k < i; ++k) s = s - at(i, k) * at(k, j);
                    at(i, j) = s;
                }
        bar.wait();
        // A22 -= L21 U12 on every thread's rows below the first half: each
        // element takes its products in k order, a column axpy per k
        own_ranges(tid, c + w1, [&](int64_t r0, int64_t r1) {
            for (int64_t j = c + w1; j < c + w; ++j) {
                double *cj = &at(0, j);
                for (int64_t k = c; k < c + w1; ++k) {
                    const double u = at(k, j);
                    const double *lk = &at(0, k);
                    for (int64_t i = r0; i < r1; ++i) cj[i] = cj[i] - lk[i] * u;
                }
            }
        });
        bar.wait();
        rec(tid, c + w1, w2);
    }
};

}  // namespace

int host_panel_factor(double *P, int64_t m, int64_t nb, int64_t ld, int32_t *ipiv, int threads, int64_t *info)
{
    if (m <= 0 || nb <= 0) {
        *info = 0;
        return HPL_OK;
    }
    const int64_t w = nb < m ? nb : m;
    HostPanel hp(P, m, nb, ld, ipiv, threads);
    std::vector<std::thread> pool;
    pool.reserve((size_t)threads - 1);
    for (int tid = 1; tid < threads; ++tid) pool.emplace_back([&hp, tid, w] { hp.rec(tid, 0, w); });
    hp.rec(0, 0, w);
    for (auto &th : pool) th.join();
    *info = hp.info;
    return HPL_OK;
}

}  // namespace hplx
