// driver.hip -- host side of libhplx: argument checks, per-device workspace,
// the blocked right-looking factorization with look-ahead, the solves, the
// residual and the generator entry points of hpl.h.
//
// Factorization loop (Sec. I / Sec. II: FACT -> RS -> UPDATE per NB-column
// panel along the diagonal; Sec. III: look-ahead).  With look-ahead on, panel
// j+1 is factored on the panel stream while the update of panel j on the
// caller's stream finishes the columns to the right of it:
//
//   update stream U                          panel stream P
//   wait panel j done
//   RS + TRSM + GEMM on panel j+1's columns  .
//   record "look-ahead done"  -------------> wait, FACT panel j+1, its plan
//   RS + TRSM + GEMM on the remaining cols   (runs concurrently)
//   RS on the columns left of panel j        record "panel j+1 done"
//
// One GPU holds the whole matrix, so the paper's LBCAST and the MPI parts of
// RS disappear: the panel's L stays in place and RS is an in-place row
// interchange.  Every element sees the same operations in the same order with
// and without look-ahead, so both give identical bits.
#include "common.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

namespace hplx {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static std::mutex g_err_mu;
static char g_err_detail[512] = "no error";

void note_hip_error(hipError_t e, const char *what, const char *file, int line)
{
    std::lock_guard<std::mutex> lk(g_err_mu);
    snprintf(g_err_detail, sizeof g_err_detail, "%s failed: %s (%d) at %s:%d", what, hipGetErrorString(e), (int)e,
             file, line);
}

void note_error(const char *what, const char *file, int line)
{
    std::lock_guard<std::mutex> lk(g_err_mu);
    snprintf(g_err_detail, sizeof g_err_detail, "%s at %s:%d", what, file, line);
}

#define HPLX_FAIL(code, what)                                                                                    \
    do {                                                                                                          \
        note_error(what, __FILE__, __LINE__);                                                                     \
        return (code);                                                                                            \
    } while (0)

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------
static std::atomic<int64_t> opt_lookahead{3};
static std::atomic<int64_t> opt_panel_base{32};
static std::atomic<int64_t> opt_panel_wgs{256};
static std::atomic<int64_t> opt_timing{0};
static std::atomic<int64_t> opt_progress{0};
static std::atomic<int64_t> opt_serialize{0};
static std::atomic<int64_t> opt_gemm_tile{0};
static std::atomic<int64_t> opt_laswp_wgs{96};
static std::atomic<int64_t> opt_host_panel{0};
static std::atomic<int64_t> opt_batch_config{0};  // 0: tuned table; else a forced schedule  // threads of the host panel (0: panel on the GPU)

// ---------------------------------------------------------------------------
// statistics (HPL_OPT_TIMING)
// ---------------------------------------------------------------------------
enum { ST_GEMM = 0, ST_PANEL = 1, ST_LASWP = 2, ST_TRSM = 3, ST_SOLVE = 4, ST_PLAN = 5, ST_MXP_GEMM = 6,
       ST_MXP_FACT = 7, ST_GRAD_A = 8, ST_BATCHED = 9, ST_N = 10 };
static std::mutex g_st_mu;
static int64_t g_st_launch[ST_N];
static double g_st_ms[ST_N], g_st_flops[ST_N], g_st_bytes[ST_N];

struct TimedRec {
    int cls;
    hipEvent_t e0, e1;
    double flops, bytes;
};

struct Device;

// A per-call list of event pairs, resolved after the call's final synchronize.
class Timer {
  public:
    explicit Timer(Device *d, bool on) : d_(d), on_(on) {}
    bool on() const { return on_; }
    int begin(int cls, hipStream_t st);
    int end(int id, hipStream_t st, double flops, double bytes);
    int collect();
    ~Timer();

  private:
    Device *d_;
    bool on_;
    std::vector<TimedRec> recs_;
};

// ---------------------------------------------------------------------------
// per-device state
// ---------------------------------------------------------------------------
constexpr int kRing = 4;        // panels in flight (plans and events are reused modulo kRing)
constexpr int kMxpMaxGroup = 32; // panels per group of the mixed-precision factorization (at most)
constexpr int kMaxChunks = 2;   // nb <= 1024 = 2 x kMaxSwaps
constexpr int kMaxDevices = 64;

struct Device {
    bool ready = false;
    int id = -1;
    hipStream_t sp = nullptr;  // panel stream (non-blocking)
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    hipEvent_t ev_panel[kRing] = {}, ev_la[kRing] = {}, ev_iter[kRing] = {};
    hipEvent_t ev_mxp[2 * kMxpMaxGroup + 1] = {};  // mixed precision look-ahead: main -> panel stream, back
    void *ws = nullptr;
    LeafSync sync{};
    unsigned long long bar_epoch = 0;
    uint32_t tag_epoch = 0;   // register-leaf tags used so far (tag 0 is never used)
    size_t tag_area_bytes = 0;
    SwapPlan ring[kRing][kMaxChunks]{};
    SwapPlan pint{};  // plans inside the recursive panel
    SwapPlan psolve{};
    unsigned long long *red = nullptr;
    int64_t red_cap = 0;
    unsigned long long *hbuf = nullptr;  // pinned host staging
    int *pivot_err = nullptr;            // raised by the plan kernel on an out-of-range pivot
    unsigned *solve_done = nullptr;      // workgroup counter of the solve's block launches (zero between them)
    int32_t *splans = nullptr;           // interchange plans of every chunk of ipiv (solve)
    int64_t splan_cap = 0;
    std::vector<hipEvent_t> ev_pool;      // timing events
    void *mxp_ws = nullptr;               // mixed precision: FP16/BF16 copies of L21 and U12, scalars
    size_t mxp_cap = 0;
    double *mxp_vec = nullptr;            // refinement vectors r, d (2 n doubles)
    int64_t mxp_vec_cap = 0;
    void *bat_ws = nullptr;               // batched systems: sizes, offsets, order, info, queue counter
    size_t bat_cap = 0;
    double *hp_buf = nullptr;             // host panel: pinned staging of the m x nb panel and its pivots
    size_t hp_cap = 0;
};

static std::mutex g_dev_mu;
static Device g_dev[kMaxDevices];

int Timer::begin(int cls, hipStream_t st)
{
    if (!on_) return -1;
    TimedRec r{cls, nullptr, nullptr, 0, 0};
    for (hipEvent_t *e : {&r.e0, &r.e1}) {
        if (!d_->ev_pool.empty()) {
            *e = d_->ev_pool.back();
            d_->ev_pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            return -1;
        }
    }
    if (hipEventRecord(r.e0, st) != hipSuccess) return -1;
    recs_.push_back(r);
    return (int)recs_.size() - 1;
}

int Timer::end(int id, hipStream_t st, double flops, double bytes)
{
    if (!on_ || id < 0) return HPL_OK;
    recs_[id].flops = flops;
    recs_[id].bytes = bytes;
    HPLX_TRY(hipEventRecord(recs_[id].e1, st));
    return HPL_OK;
}

int Timer::collect()
{
    if (!on_) return HPL_OK;
    std::lock_guard<std::mutex> lk(g_st_mu);
    for (auto &r : recs_) {
        float ms = 0.f;
        HPLX_TRY(hipEventElapsedTime(&ms, r.e0, r.e1));
        g_st_launch[r.cls] += 1;
        g_st_ms[r.cls] += ms;
        g_st_flops[r.cls] += r.flops;
        g_st_bytes[r.cls] += r.bytes;
    }
    return HPL_OK;
}

Timer::~Timer()
{
    for (auto &r : recs_) {
        d_->ev_pool.push_back(r.e0);
        d_->ev_pool.push_back(r.e1);
    }
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int init_device(Device &d, int id)
{
    hipDeviceProp_t prop;
    HPLX_TRY(hipGetDeviceProperties(&prop, id));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) HPLX_FAIL(HPL_ERR_DEVICE, "device is not gfx950");
    HPLX_TRY(hipStreamCreateWithFlags(&d.sp, hipStreamNonBlocking));
    HPLX_TRY(hipEventCreateWithFlags(&d.ev_start, hipEventDisableTiming));
    HPLX_TRY(hipEventCreateWithFlags(&d.ev_end, hipEventDisableTiming));
    for (int i = 0; i < kRing; ++i) {
        HPLX_TRY(hipEventCreateWithFlags(&d.ev_panel[i], hipEventDisableTiming));
        HPLX_TRY(hipEventCreateWithFlags(&d.ev_la[i], hipEventDisableTiming));
        HPLX_TRY(hipEventCreateWithFlags(&d.ev_iter[i], hipEventDisableTiming));
    }
    for (hipEvent_t &e : d.ev_mxp) HPLX_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // one workspace block: sync words, leaf slots, interchange plans
    const size_t plan_bytes = align_up(2 * kMaxSwaps * sizeof(int32_t), 256) * 2 + 256;
    size_t o = 0;
    const size_t o_ctr = o; o += 256;
    const size_t o_abort = o; o += 256;
    const size_t o_info = o; o += 256;
    const size_t o_perr = o; o += 256;
    const size_t o_sdone = o; o += 256;
    const size_t o_slots = o; o = align_up(o + sizeof(double) * 2 * kLeafMaxWGs * kLeafSlot, 256);
    const size_t o_top = o; o = align_up(o + sizeof(double) * 2 * kLeafMaxW, 256);
    const size_t o_tslots = o; o = align_up(o + sizeof(unsigned long long) * 2 * kLeafMaxWGs * kLeafSlotWords, 256);
    const size_t o_ttop = o; o = align_up(o + sizeof(unsigned long long) * 2 * 64, 256);
    d.tag_area_bytes = o - o_tslots;
    const size_t o_plans = o; o += plan_bytes * (kRing * kMaxChunks + 2);
    void *ws = nullptr;
    if (hipMalloc(&ws, o) != hipSuccess) HPLX_FAIL(HPL_ERR_NOMEM, "workspace allocation failed");
    d.ws = ws;
    char *b = (char *)ws;
    d.sync.counter = (unsigned long long *)(b + o_ctr);
    d.sync.abort_flag = (int *)(b + o_abort);
    d.sync.info = (unsigned long long *)(b + o_info);
    d.pivot_err = (int *)(b + o_perr);
    d.solve_done = (unsigned *)(b + o_sdone);
    d.sync.slots = (double *)(b + o_slots);
    d.sync.top = (double *)(b + o_top);
    d.sync.tslots = (unsigned long long *)(b + o_tslots);
    d.sync.ttop = (unsigned long long *)(b + o_ttop);
    auto plan_at = [&](int k) {
        char *p = b + o_plans + (size_t)k * plan_bytes;
        SwapPlan s;
        s.rows = (int32_t *)p;
        s.srcslot = (int32_t *)(p + align_up(2 * kMaxSwaps * sizeof(int32_t), 256));
        s.nslots = (int32_t *)(p + 2 * align_up(2 * kMaxSwaps * sizeof(int32_t), 256));
        s.err = (int *)(b + o_perr);
        return s;
    };
    for (int r = 0; r < kRing; ++r)
        for (int q = 0; q < kMaxChunks; ++q) d.ring[r][q] = plan_at(r * kMaxChunks + q);
    d.pint = plan_at(kRing * kMaxChunks);
    d.psolve = plan_at(kRing * kMaxChunks + 1);
    HPLX_TRY(hipMemset(ws, 0, o));
    HPLX_TRY(hipHostMalloc((void **)&d.hbuf, 4096, hipHostMallocDefault));
    HPLX_TRY(hipDeviceSynchronize());
    d.bar_epoch = 0;
    d.id = id;
    d.ready = true;
    return HPL_OK;
}

static int get_device(Device **out)
{
    int id = 0;
    HPLX_TRY(hipGetDevice(&id));
    if (id < 0 || id >= kMaxDevices) HPLX_FAIL(HPL_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    Device &d = g_dev[id];
    if (!d.ready) {
        int rc = init_device(d, id);
        if (rc != HPL_OK) return rc;
    }
    *out = &d;
    return HPL_OK;
}

static int ensure_red(Device *d, int64_t count)
{
    if (d->red_cap >= count) return HPL_OK;
    if (d->red) HPLX_TRY(hipFree(d->red));
    d->red = nullptr;
    d->red_cap = 0;
    if (hipMalloc((void **)&d->red, sizeof(unsigned long long) * count) != hipSuccess)
        HPLX_FAIL(HPL_ERR_NOMEM, "residual buffer allocation failed");
    d->red_cap = count;
    return HPL_OK;
}

// ---------------------------------------------------------------------------
// building blocks
// ---------------------------------------------------------------------------
struct Ctx {
    Device *d;
    double *A;
    int64_t n, lda;
    int32_t *ipiv;
    int base, gmax, gemm_tile;
    Timer *tm;
    int host_threads = 0;       // > 0: the panel is factored on the host (the paper's CPU FACT)
    int64_t host_info = 0;      // first zero pivot (1-based) found by the host panel
};

// Interchange plans of ipiv[k0 .. k0+cnt) (cnt <= kMaxChunks*kMaxSwaps) into plans[].
static int make_plans(const int32_t *ipiv_k0, int64_t k0, int64_t cnt, int64_t nrows, SwapPlan *plans,
                      bool reverse, hipStream_t st, Timer *tm)
{
    int id = tm->begin(ST_PLAN, st);
    for (int64_t q = 0; q * kMaxSwaps < cnt; ++q) {
        const int64_t off0 = q * kMaxSwaps;
        const int64_t c = (cnt - off0) < kMaxSwaps ? (cnt - off0) : kMaxSwaps;
        HPLX_PROPAGATE(launch_swap_plan(ipiv_k0 + off0, (int)c, k0 + off0, nrows, reverse, plans[q], st));
    }
    return tm->end(id, st, 0, 0);
}

static int apply_plans(double *A, int64_t lda, int64_t col0, int64_t ncols, int64_t cnt, SwapPlan *plans,
                       hipStream_t st, Timer *tm)
{
    if (ncols <= 0 || cnt <= 0) return HPL_OK;
    int id = tm->begin(ST_LASWP, st);
    const int64_t max_wgs = opt_laswp_wgs.load();
    for (int64_t q = 0; q * kMaxSwaps < cnt; ++q)
        HPLX_PROPAGATE(launch_laswp(A, lda, col0, ncols, plans[q], max_wgs, st));
    return tm->end(id, st, 0, 32.0 * (double)cnt * (double)ncols);
}

// B(nbk x ncols) <- L^{-1} B for nbk <= 1024 (row chunks of 512 joined by a GEMM).
static int trsm_any(const double *L, int64_t ldl, double *B, int64_t ldb, int64_t nbk, int64_t ncols, int tile,
                    hipStream_t st)
{
    if (nbk <= 512) return launch_trsm_llnu(L, ldl, B, ldb, nbk, ncols, st);
    HPLX_PROPAGATE(launch_trsm_llnu(L, ldl, B, ldb, 512, ncols, st));
    HPLX_PROPAGATE(launch_gemm_sub(nbk - 512, ncols, 512, L + 512, ldl, B, ldb, B + 512, ldb, tile, st));
    return launch_trsm_llnu(L + off(512, 512, ldl), ldl, B + 512, ldb, nbk - 512, ncols, st);
}

// Recursive panel factorization of columns [c, c+w), rows [c, n) (Sec. III-A:
// recursive right-looking, two halves per level, small leaves factored
// right-looking).
static int panel_rec(Ctx &x, int64_t c, int64_t w, hipStream_t st)
{
    Device *d = x.d;
    if (w <= x.base) {
        const int64_t m = x.n - c;
        const int Gr = leaf_reg_groups(m, (int)w);
        if (Gr > 0 && Gr <= x.gmax) {
            if (d->tag_epoch > 0xF0000000u) {  // far from wrapping: clear the words, restart the tags
                HPLX_PROPAGATE(launch_fill_u64(d->sync.tslots, (int64_t)(d->tag_area_bytes / 8), 0ull, st));
                d->tag_epoch = 0;
            }
            const uint32_t tag0 = d->tag_epoch;
            d->tag_epoch += (uint32_t)w + 1u;
            return launch_leaf_reg(x.A, x.lda, c, m, (int)w, x.ipiv, d->sync, tag0, Gr, st);
        }
        const int G = leaf_groups(m, (int)w, x.gmax);
        const unsigned long long base_ctr = d->bar_epoch;
        if (G > 1) d->bar_epoch += (unsigned long long)G * (unsigned long long)w;
        return launch_panel_leaf(x.A, x.lda, c, m, (int)w, x.ipiv, d->sync, base_ctr, G, st);
    }
    int64_t w1 = ((w / 2 + x.base - 1) / x.base) * x.base;
    if (w1 >= w) w1 = w - 1;
    const int64_t w2 = w - w1;
    HPLX_PROPAGATE(panel_rec(x, c, w1, st));
    HPLX_PROPAGATE(launch_swap_plan(x.ipiv + c, (int)w1, c, x.n, false, d->pint, st));
    HPLX_PROPAGATE(launch_laswp(x.A, x.lda, c + w1, w2, d->pint, 0, st));
    HPLX_PROPAGATE(launch_trsm_llnu(x.A + off(c, c, x.lda), x.lda, x.A + off(c, c + w1, x.lda), x.lda, w1, w2, st));
    if (gemm_skinny_ok(w2, w1))
        HPLX_PROPAGATE(launch_gemm_skinny(x.n - c - w1, w2, w1, x.A + off(c + w1, c, x.lda), x.lda,
                                          x.A + off(c, c + w1, x.lda), x.lda, x.A + off(c + w1, c + w1, x.lda), x.lda,
                                          st));
    else
        HPLX_PROPAGATE(launch_gemm_sub(x.n - c - w1, w2, w1, x.A + off(c + w1, c, x.lda), x.lda,
                                       x.A + off(c, c + w1, x.lda), x.lda, x.A + off(c + w1, c + w1, x.lda), x.lda,
                                       0, st));
    HPLX_PROPAGATE(panel_rec(x, c + w1, w2, st));
    HPLX_PROPAGATE(launch_swap_plan(x.ipiv + c + w1, (int)w2, c + w1, x.n, false, d->pint, st));
    return launch_laswp(x.A, x.lda, c, w1, d->pint, 0, st);
}

static int panel_full(Ctx &x, int64_t c0, int64_t jb, SwapPlan *plans, hipStream_t st)
{
    const double m = (double)(x.n - c0);
    const double w = (double)jb;
    int id = x.tm->begin(ST_PANEL, st);
    HPLX_PROPAGATE(panel_rec(x, c0, jb, st));
    // flops of LU of an m x w panel: m w^2 - w^3/3 (plus lower-order terms)
    HPLX_PROPAGATE(x.tm->end(id, st, m * w * w - w * w * w / 3.0, 16.0 * m * w));
    return make_plans(x.ipiv + c0, c0, jb, x.n, plans, false, st, x.tm);
}

// FACT of panel (c0, jb) on the host (the paper's CPU FACT, Sec. III-A): the
// panel goes to pinned host memory once its columns are up to date in the
// order of stream st, T threads factor it, and the factors and pivots return
// on st, followed by the interchange plans.  The calling thread blocks for
// the copy out and the factorization; work queued earlier on other streams
// keeps the GPU busy meanwhile.
static int panel_host(Ctx &x, int64_t c0, int64_t jb, SwapPlan *plans, hipStream_t st)
{
    Device *d = x.d;
    const int64_t m = x.n - c0;
    const size_t need = sizeof(double) * (size_t)m * (size_t)jb + sizeof(int32_t) * (size_t)jb + 64;
    if (d->hp_cap < need) {
        if (d->hp_buf) HPLX_TRY(hipHostFree(d->hp_buf));
        d->hp_buf = nullptr;
        d->hp_cap = 0;
        const size_t cap = sizeof(double) * (size_t)x.n * (size_t)jb + sizeof(int32_t) * (size_t)jb + 64;
        if (hipHostMalloc((void **)&d->hp_buf, cap, hipHostMallocDefault) != hipSuccess)
            HPLX_FAIL(HPL_ERR_NOMEM, "host panel staging allocation failed");
        d->hp_cap = cap;
    }
    double *P = d->hp_buf;
    int32_t *hip_piv = (int32_t *)(P + (size_t)m * (size_t)jb);
    double *src = x.A + off(c0, c0, x.lda);
    HPLX_TRY(hipMemcpy2DAsync(P, sizeof(double) * (size_t)m, src, sizeof(double) * (size_t)x.lda,
                              sizeof(double) * (size_t)m, (size_t)jb, hipMemcpyDeviceToHost, st));
    const auto th0 = std::chrono::steady_clock::now();
    HPLX_TRY(hipStreamSynchronize(st));
    int64_t inf = 0;
    HPLX_PROPAGATE(host_panel_factor(P, m, jb, m, hip_piv, x.host_threads, &inf));
    if (opt_timing.load()) {  // the panel class: copy out + host FACT, wall time
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
        const double mm = (double)m, w = (double)jb;
        std::lock_guard<std::mutex> lk(g_st_mu);
        g_st_launch[ST_PANEL] += 1;
        g_st_ms[ST_PANEL] += ms;
        g_st_flops[ST_PANEL] += mm * w * w - w * w * w / 3.0;
        g_st_bytes[ST_PANEL] += 16.0 * mm * w;
    }
    if (inf > 0 && (x.host_info == 0 || c0 + inf < x.host_info)) x.host_info = c0 + inf;
    for (int64_t k = 0; k < jb; ++k) hip_piv[k] += (int32_t)c0;
    HPLX_TRY(hipMemcpy2DAsync(src, sizeof(double) * (size_t)x.lda, P, sizeof(double) * (size_t)m,
                              sizeof(double) * (size_t)m, (size_t)jb, hipMemcpyHostToDevice, st));
    HPLX_TRY(hipMemcpyAsync(x.ipiv + c0, hip_piv, sizeof(int32_t) * (size_t)jb, hipMemcpyHostToDevice, st));
    return make_plans(x.ipiv + c0, c0, jb, x.n, plans, false, st, x.tm);
}

static int panel_any(Ctx &x, int64_t c0, int64_t jb, SwapPlan *plans, hipStream_t st)
{
    return x.host_threads > 0 ? panel_host(x, c0, jb, plans, st) : panel_full(x, c0, jb, plans, st);
}

// Trailing GEMM of panel (c0, jb) on columns [col, col+ncols): A22 -= L21 U12.
static int update_gemm(Ctx &x, int64_t c0, int64_t jb, int64_t col, int64_t ncols, hipStream_t st)
{
    const int64_t c1 = c0 + jb;
    const int64_t m = x.n - c1;
    if (m <= 0 || ncols <= 0) return HPL_OK;
    int id = x.tm->begin(ST_GEMM, st);
    HPLX_PROPAGATE(launch_gemm_sub(m, ncols, jb, x.A + off(c1, c0, x.lda), x.lda, x.A + off(c0, col, x.lda), x.lda,
                                   x.A + off(c1, col, x.lda), x.lda, x.gemm_tile | kGemmTrailing, st));
    return x.tm->end(id, st, 2.0 * (double)m * (double)ncols * (double)jb,
                     16.0 * (double)m * (double)ncols + 8.0 * (double)jb * ((double)m + (double)ncols));
}

// RS + TRSM (+ GEMM when with_gemm) of panel (c0, jb) applied to columns [col, col+ncols).
static int update_cols(Ctx &x, int64_t c0, int64_t jb, int64_t col, int64_t ncols, SwapPlan *plans, hipStream_t st,
                       bool with_gemm)
{
    if (ncols <= 0) return HPL_OK;
    HPLX_PROPAGATE(apply_plans(x.A, x.lda, col, ncols, jb, plans, st, x.tm));
    int id = x.tm->begin(ST_TRSM, st);
    HPLX_PROPAGATE(trsm_any(x.A + off(c0, c0, x.lda), x.lda, x.A + off(c0, col, x.lda), x.lda, jb, ncols,
                            x.gemm_tile, st));
    HPLX_PROPAGATE(x.tm->end(id, st, (double)jb * (double)jb * (double)ncols, 16.0 * (double)jb * (double)ncols));
    return with_gemm ? update_gemm(x, c0, jb, col, ncols, st) : HPL_OK;
}

// Reports (and clears) an out-of-range pivot seen by the plan kernel; hbuf[2] holds the flag.
static int check_pivot_error(Device *d, hipStream_t st)
{
    if (*(int *)(d->hbuf + 2) == 0) return HPL_OK;
    HPLX_TRY(hipMemsetAsync(d->pivot_err, 0, sizeof(int), st));
    HPLX_TRY(hipStreamSynchronize(st));
    HPLX_FAIL(HPL_ERR_INTERNAL, "pivot index outside [k, n) in ipiv");
}

static double now_s()
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

// LU of the n x n matrix in A's first n columns.  nextra > 0: the columns
// [n, n + nextra) are right-hand sides carried along as part of an augmented
// system (every panel's interchanges, TRSM and GEMM reach them like any other
// trailing column, so they end as L^{-1} P^{-1} B).  left_swaps: each panel's
// interchanges are also applied to the columns left of it (L in LAPACK form);
// without, each panel's multipliers stay in the row order of their own
// factorization, as in HPL, where the row swaps reach only the columns to the
// right of the panel (Sec. II).
static int factor_impl(Device *d, double *A, int64_t n, int64_t lda, int64_t nb, int32_t *ipiv, int64_t *info,
                       hipStream_t su, int64_t nextra = 0, bool left_swaps = true)
{
    const int64_t ncol = n + nextra;
    Timer tm(d, opt_timing.load() != 0);
    Ctx x{d, A, n, lda, ipiv, (int)opt_panel_base.load(), (int)opt_panel_wgs.load(), (int)opt_gemm_tile.load(), &tm};
    x.host_threads = (int)opt_host_panel.load();
    const int64_t progress = opt_progress.load();
    // mode 3 (the default) takes 2 up to n = 32768, where the panel is the
    // critical path and the small trailing GEMMs leave it CUs, else 1
    const int64_t la_opt = opt_lookahead.load();
    const int64_t la_mode = la_opt == 3 ? (n <= 32768 ? 2 : 1) : la_opt;
    const bool la = la_mode != 0 && opt_serialize.load() == 0 && n > nb;
    hipStream_t sp = la ? d->sp : su;
    const int64_t np = (n + nb - 1) / nb;
    const double t0 = now_s();

    HPLX_PROPAGATE(launch_fill_u64(d->sync.info, 1, ULLONG_MAX, su));
    if (la) {
        HPLX_TRY(hipEventRecord(d->ev_start, su));
        HPLX_TRY(hipStreamWaitEvent(sp, d->ev_start, 0));
    }
    HPLX_PROPAGATE(panel_any(x, 0, nb < n ? nb : n, d->ring[0], sp));
    if (la) HPLX_TRY(hipEventRecord(d->ev_panel[0], sp));

    for (int64_t j = 0; j < np; ++j) {
        const int64_t c0 = j * nb;
        const int64_t jb = (n - c0) < nb ? (n - c0) : nb;
        const int64_t c1 = c0 + jb;
        SwapPlan *plans = d->ring[j % kRing];
        bool left_done = false;
        if (la) HPLX_TRY(hipStreamWaitEvent(su, d->ev_panel[j % kRing], 0));
        if (c1 < n) {
            const int64_t jb2 = (n - c1) < nb ? (n - c1) : nb;
            SwapPlan *next_plans = d->ring[(j + 1) % kRing];
            if (la && x.host_threads > 0) {
                // host FACT (the paper's scheme): the whole rest of the update,
                // GEMM included, is queued first and overlaps the host work;
                // the next iteration waits for the panel's event
                HPLX_PROPAGATE(update_cols(x, c0, jb, c1, jb2, plans, su, true));
                HPLX_TRY(hipEventRecord(d->ev_la[j % kRing], su));
                HPLX_PROPAGATE(update_cols(x, c0, jb, c1 + jb2, ncol - c1 - jb2, plans, su, true));
                if (left_swaps) HPLX_PROPAGATE(apply_plans(A, lda, 0, c0, jb, plans, su, &tm));
                left_done = true;
                HPLX_TRY(hipStreamWaitEvent(sp, d->ev_la[j % kRing], 0));
                HPLX_PROPAGATE(panel_host(x, c1, jb2, next_plans, sp));
                HPLX_TRY(hipEventRecord(d->ev_panel[(j + 1) % kRing], sp));
            } else if (la) {
                HPLX_PROPAGATE(update_cols(x, c0, jb, c1, jb2, plans, su, true));
                HPLX_TRY(hipEventRecord(d->ev_la[j % kRing], su));
                HPLX_TRY(hipStreamWaitEvent(sp, d->ev_la[j % kRing], 0));
                HPLX_PROPAGATE(panel_full(x, c1, jb2, next_plans, sp));
                HPLX_TRY(hipEventRecord(d->ev_panel[(j + 1) % kRing], sp));
                if (la_mode == 2) {
                    // full overlap: the trailing GEMM shares the GPU with the panel
                    HPLX_PROPAGATE(update_cols(x, c0, jb, c1 + jb2, ncol - c1 - jb2, plans, su, true));
                } else {
                    // the panel overlaps the memory-bound RS and TRSM of the
                    // remaining columns and the interchanges on the left; the
                    // trailing GEMM starts once the panel is done, so the two
                    // never compete for the CUs
                    HPLX_PROPAGATE(update_cols(x, c0, jb, c1 + jb2, ncol - c1 - jb2, plans, su, false));
                    if (left_swaps) HPLX_PROPAGATE(apply_plans(A, lda, 0, c0, jb, plans, su, &tm));
                    left_done = true;
                    HPLX_TRY(hipStreamWaitEvent(su, d->ev_panel[(j + 1) % kRing], 0));
                    HPLX_PROPAGATE(update_gemm(x, c0, jb, c1 + jb2, ncol - c1 - jb2, su));
                }
            } else {
                HPLX_PROPAGATE(update_cols(x, c0, jb, c1, ncol - c1, plans, su, true));
                HPLX_PROPAGATE(panel_any(x, c1, jb2, next_plans, su));
            }
        } else if (nextra > 0) {
            // last panel: its interchanges and L11^{-1} reach the carried columns
            HPLX_PROPAGATE(update_cols(x, c0, jb, n, nextra, plans, su, true));
        }
        // interchanges of panel j on the columns to its left (L in LAPACK form)
        if (!left_done && left_swaps) HPLX_PROPAGATE(apply_plans(A, lda, 0, c0, jb, plans, su, &tm));
        HPLX_TRY(hipEventRecord(d->ev_iter[j % kRing], su));
        // keep at most two iterations queued ahead of the device
        if (j >= 2) HPLX_TRY(hipEventSynchronize(d->ev_iter[(j - 2) % kRing]));
        if (progress > 0 && ((j + 1) % progress == 0 || j + 1 == np)) {
            fprintf(stderr, "[hplx] panel %lld/%lld queued, %.2f s\n", (long long)(j + 1), (long long)np,
                    now_s() - t0);
            fflush(stderr);
        }
    }
    HPLX_TRY(hipMemcpyAsync(d->hbuf, d->sync.info, sizeof(unsigned long long), hipMemcpyDeviceToHost, su));
    HPLX_TRY(hipMemcpyAsync(d->hbuf + 1, d->sync.abort_flag, sizeof(int), hipMemcpyDeviceToHost, su));
    HPLX_TRY(hipMemcpyAsync(d->hbuf + 2, d->pivot_err, sizeof(int), hipMemcpyDeviceToHost, su));
    HPLX_TRY(hipStreamSynchronize(su));
    if (la) HPLX_TRY(hipStreamSynchronize(sp));
    HPLX_PROPAGATE(tm.collect());
    HPLX_PROPAGATE(check_pivot_error(d, su));
    const int aborted = *(int *)(d->hbuf + 1);
    if (aborted) {
        HPLX_PROPAGATE(launch_fill_u64(d->sync.counter, 1, 0ull, su));
        HPLX_PROPAGATE(launch_fill_u64(d->sync.tslots, (int64_t)(d->tag_area_bytes / 8), 0ull, su));
        HPLX_TRY(hipMemsetAsync(d->sync.abort_flag, 0, sizeof(int), su));
        HPLX_TRY(hipStreamSynchronize(su));
        d->bar_epoch = 0;
        d->tag_epoch = 0;
        HPLX_FAIL(HPL_ERR_INTERNAL, "panel barrier timed out");
    }
    const unsigned long long iv = d->hbuf[0];
    int64_t inf = (iv == ULLONG_MAX) ? 0 : (int64_t)iv;
    if (x.host_info > 0 && (inf == 0 || x.host_info < inf)) inf = x.host_info;
    *info = inf;
    return HPL_OK;
}

static int ensure_solve_plans(Device *d, int64_t nchunks)
{
    if (d->splan_cap >= nchunks) return HPL_OK;
    if (d->splans) HPLX_TRY(hipFree(d->splans));
    d->splans = nullptr;
    d->splan_cap = 0;
    if (hipMalloc((void **)&d->splans, sizeof(int32_t) * (size_t)kPlanStride * (size_t)nchunks) != hipSuccess)
        HPLX_FAIL(HPL_ERR_NOMEM, "solve plan buffer allocation failed");
    d->splan_cap = nchunks;
    return HPL_OK;
}

static int solve_impl(Device *d, const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n,
                      int64_t lda, int64_t ldb, int trans, hipStream_t st)
{
    Timer tm(d, opt_timing.load() != 0);
    const int64_t nchunks = (n + kMaxSwaps - 1) / kMaxSwaps;
    HPLX_PROPAGATE(ensure_solve_plans(d, nchunks));
    int id = tm.begin(ST_SOLVE, st);
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)d->solve_done, 1, 0ull, st));
    HPLX_PROPAGATE(solve_sequence(LU, ipiv, B, nrhs, n, lda, ldb, trans, d->splans, d->pivot_err, d->solve_done, st));
    HPLX_PROPAGATE(tm.end(id, st, 2.0 * (double)n * (double)n * (double)nrhs, 8.0 * (double)n * (double)n));
    HPLX_TRY(hipMemcpyAsync(d->hbuf + 2, d->pivot_err, sizeof(int), hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    HPLX_PROPAGATE(tm.collect());
    return check_pivot_error(d, st);
}

// ---------------------------------------------------------------------------
// mixed precision (no pivoting; FP32 working matrix; FP16/BF16 trailing update)
// ---------------------------------------------------------------------------
static int ensure_mxp_ws(Device *d, size_t bytes)
{
    if (d->mxp_cap >= bytes) return HPL_OK;
    if (d->mxp_ws) HPLX_TRY(hipFree(d->mxp_ws));
    d->mxp_ws = nullptr;
    d->mxp_cap = 0;
    if (hipMalloc(&d->mxp_ws, bytes) != hipSuccess) HPLX_FAIL(HPL_ERR_NOMEM, "mixed-precision workspace allocation failed");
    d->mxp_cap = bytes;
    return HPL_OK;
}

// B (nbk x ncols) <- L^{-1} B, L unit lower (FP32): 64-row leaves joined by
// GEMMs.  With mx, the largest |value| of the solution is folded into *mx (by
// the leaves, which store final values).
static int mxp_trsm(const float *L, int64_t ldl, int64_t nbk, float *B, int64_t ldb, int64_t ncols, hipStream_t st,
                    unsigned *mx = nullptr)
{
    if (nbk <= 0 || ncols <= 0) return HPL_OK;
    if (nbk <= kTrsm32LeafMax) return launch_trsm32_leaf(L, ldl, B, ldb, (int)nbk, ncols, st, mx);
    // the panel's own solves (few columns): one launch instead of a recursion
    // of leaves and GEMMs
    if (trsm32_small_ok(nbk, ncols)) return launch_trsm32_small(L, ldl, B, ldb, nbk, ncols, st, mx);
    const int64_t h = ((nbk / 2 + 31) / 32) * 32;
    HPLX_PROPAGATE(mxp_trsm(L, ldl, h, B, ldb, ncols, st, mx));
    HPLX_PROPAGATE(launch_sgemm32(nbk - h, ncols, h, L + h, ldl, B, ldb, B + h, ldb, st));
    return mxp_trsm(L + off(h, h, ldl), ldl, nbk - h, B + h, ldb, ncols, st, mx);
}

// FACT of columns [c, c+w), rows [c, n), no pivoting, FP32: recursive halves.
// With mx, the largest |l| of the rows from l21_row0 on is folded into *mx
// (by the leaves, which store final values).
static int mxp_panel(float *A, int64_t lda, int64_t n, int64_t c, int64_t w, unsigned long long *info, unsigned *done,
                     hipStream_t st, unsigned *mx = nullptr, int64_t l21_row0 = 0)
{
    if (w <= kPanel32LeafMax) return launch_panel32_leaf(A, lda, c, n, (int)w, info, done, st, mx, l21_row0);
    int64_t w1 = ((w / 2 + 31) / 32) * 32;
    if (w1 >= w) w1 = w - 1;
    const int64_t w2 = w - w1;
    HPLX_PROPAGATE(mxp_panel(A, lda, n, c, w1, info, done, st, mx, l21_row0));
    HPLX_PROPAGATE(mxp_trsm(A + off(c, c, lda), lda, w1, A + off(c, c + w1, lda), lda, w2, st));
    HPLX_PROPAGATE(launch_sgemm32(n - c - w1, w2, w1, A + off(c + w1, c, lda), lda, A + off(c, c + w1, lda), lda,
                                  A + off(c + w1, c + w1, lda), lda, st));
    return mxp_panel(A, lda, n, c + w1, w2, info, done, st, mx, l21_row0);
}

// The mixed-precision factorization takes the panels in groups of G (G nb =
// kMxpJoint columns: G = 2 at nb = 1024).  Per panel: FACT (FP32), U12 =
// L11^{-1} A12 (FP32), the scaling and conversion of -L21 and U12 to
// FP16/BF16.  Inside a group, panel i's columns and rows take the updates of
// panels 0 .. i-1 of the group (k = i nb) just before its FACT and its U12;
// the rest of the trailing matrix takes the update of the whole group at once,
// A22 += [-L21(0) .. -L21(G-1)] [U12(0); ..; U12(G-1)] with k = G nb: the FP32
// trailing matrix is read and written once per G panels instead of once per
// panel (the same products; only their FP32 sum over the group is rounded
// once more before it meets A22).  The operand copies of a group sit side by
// side in k in one buffer (panel i in k slots [i nb, (i+1) nb)), indexed from
// the first row (column) below (right of) the group's panel 0.
//
// With look-ahead (Sec. III) the group's joint update does, in order, the
// columns then the rows of each panel of the next group, then the rest; the
// panel stream takes each panel of the next group (its update by the group's
// earlier panels, FACT, U12 and copies into the second buffer) as soon as the
// joint update has reached its columns and rows, all beside the bulk of the
// joint update; the next group starts when both streams are done.  Every
// element takes the same operations in the same order either way (the two
// update kernels round alike), so the factors are bitwise equal.
constexpr int64_t kMxpJoint = 2048;  // k of the joint update of a group (G nb)
static int mxp_factor_impl(Device *d, const double *A, int64_t n, int64_t lda, int64_t nb, int fmt, float *LU,
                           int64_t ldlu, int64_t *info, hipStream_t st)
{
    const bool la = opt_lookahead.load() != 0 && opt_serialize.load() == 0 && n > nb;
    int64_t G = kMxpJoint / nb;
    if (G < 1) G = 1;
    if (G > kMxpMaxGroup) G = kMxpMaxGroup;
    const int64_t gw = G * nb;  // columns per group, k of the joint update
    // a buffer holds gw k for rows (columns) 0 .. n-1 below the group's panel 0
    const int64_t ss = (n + 15) / 16 * 512;  // slab stride, elements
    const size_t half_bytes = (sizeof(uint16_t) * (size_t)ss * (size_t)(gw / 32) + 255) / 256 * 256;
    const int nbuf = la ? 2 : 1;
    const size_t sc_off = 2 * (size_t)nbuf * half_bytes;
    HPLX_PROPAGATE(ensure_mxp_ws(d, sc_off + 256));
    char *ws = (char *)d->mxp_ws;
    uint16_t *A16[2], *B16[2];
    for (int q = 0; q < 2; ++q) {
        const int qq = q < nbuf ? q : 0;
        A16[q] = (uint16_t *)(ws + 2 * (size_t)qq * half_bytes);
        B16[q] = (uint16_t *)(ws + (2 * (size_t)qq + 1) * half_bytes);
    }
    // two pairs of maxima (|L21|, |U12|), used by alternate panels: a panel's
    // conversion clears the other pair for the next panel
    unsigned *mx = (unsigned *)(ws + sc_off);
    int prep_count = 0;
    unsigned long long *dinfo = (unsigned long long *)(ws + sc_off + 32);
    unsigned *leaf_done = (unsigned *)(ws + sc_off + 64);  // panel leaf's workgroup count (returns to zero)
    hipStream_t sp = la ? d->sp : st;
    Timer tm(d, opt_timing.load() != 0);
    // FACT of the panel at c (width w), on stream s; its leaves fold max |L21|
    // into the pair of maxima its conversion will use
    auto fact = [&](int64_t c, int64_t w, hipStream_t s) -> int {
        const int id = tm.begin(ST_MXP_FACT, s);
        HPLX_PROPAGATE(mxp_panel(LU, ldlu, n, c, w, dinfo, leaf_done, s, mx + 2 * (prep_count & 1), c + w));
        return tm.end(id, s, (double)(n - c) * (double)w * (double)w, 4.0 * (double)(n - c) * (double)w * 2.0);
    };
    // U12 of the panel at c (width nb) and the low-precision copies of -L21 and
    // U12 into buffer q, rows (columns) from index idx and k from slot i, on s
    auto prep = [&](int64_t c, int q, int64_t idx, int64_t i, hipStream_t s) -> int {
        const int64_t c1 = c + nb, m = n - c1;
        const size_t o = (size_t)i * (size_t)(nb / 32) * (size_t)ss + (size_t)(idx / 16) * 512;
        const int id = tm.begin(ST_MXP_FACT, s);
        // max |U12| folded into pm[1] by the solve's leaves (max |L21| is in
        // pm[0] from the panel's FACT)
        unsigned *pm = mx + 2 * (prep_count & 1), *other = mx + 2 * ((prep_count + 1) & 1);
        ++prep_count;
        HPLX_PROPAGATE(mxp_trsm(LU + off(c, c, ldlu), ldlu, nb, LU + off(c, c1, ldlu), ldlu, m, s, pm + 1));
        HPLX_PROPAGATE(launch_mxp_convert(fmt, LU + off(c1, c, ldlu), ldlu, m, LU + off(c, c1, ldlu), ldlu, m, (int)nb,
                                          pm, other, A16[q] + o, ss, B16[q] + o, ss, s));
        return tm.end(id, s, (double)nb * (double)nb * (double)m, 4.0 * (double)nb * (double)m * 2.0);
    };
    // A22 rows [b0 + i0, b0 + i0 + ni) x columns [b0 + j0, b0 + j0 + nc) += the
    // product of k = K of buffer q (b0 = the first row below the group's panel 0), on s
    auto update = [&](int64_t b0, int q, int64_t i0, int64_t ni, int64_t j0, int64_t nc, int64_t K,
                      hipStream_t s) -> int {
        if (ni <= 0 || nc <= 0) return HPL_OK;
        const int id = tm.begin(ST_MXP_GEMM, s);
        HPLX_PROPAGATE(launch_hgemm_update(fmt, ni, nc, K, A16[q] + (size_t)(i0 / 16) * 512, ss,
                                           B16[q] + (size_t)(j0 / 16) * 512, ss, LU + off(b0 + i0, b0 + j0, ldlu),
                                           ldlu, s));
        return tm.end(id, s, 2.0 * (double)ni * (double)nc * (double)K,
                      8.0 * (double)ni * (double)nc + 2.0 * (double)K * (double)(ni + nc));
    };
    // the panel work of the group at c into buffer q, on stream s, its panel 0
    // factored; with look-ahead, panel i first waits for the joint update of
    // the previous group to reach its columns (ev[2i]) and its rows (ev[2i+1])
    auto group_panels = [&](int64_t c, int q, hipStream_t s, hipEvent_t *ev) -> int {
        const int64_t b0 = c + nb;
        for (int64_t i = 0; i < G; ++i) {
            const int64_t ci = c + i * nb;  // panel i
            if (ci >= n) break;
            const int64_t wi = (n - ci) < nb ? (n - ci) : nb;
            if (i > 0) {
                if (ev) HPLX_TRY(hipStreamWaitEvent(s, ev[2 * i], 0));
                HPLX_PROPAGATE(update(b0, q, ci - b0, n - ci, ci - b0, wi, i * nb, s));  // its columns
                HPLX_PROPAGATE(fact(ci, wi, s));
            }
            if (ci + wi >= n) break;  // the last panel of the matrix
            if (ev) HPLX_TRY(hipStreamWaitEvent(s, ev[2 * i + 1], 0));
            if (i > 0) HPLX_PROPAGATE(update(b0, q, ci - b0, wi, ci + wi - b0, n - ci - wi, i * nb, s));  // its rows
            HPLX_PROPAGATE(prep(ci, q, ci + wi - b0, i, s));
        }
        return HPL_OK;
    };
    HPLX_PROPAGATE(launch_fill_u64(dinfo, 1, ULLONG_MAX, st));
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)leaf_done, 1, 0ull, st));
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)mx, 2, 0ull, st));
    HPLX_PROPAGATE(launch_cvt_f64_f32(A, lda, LU, ldlu, n, n, st));
    HPLX_PROPAGATE(fact(0, nb < n ? nb : n, st));
    int cur = 0;
    if (nb < n) HPLX_PROPAGATE(group_panels(0, cur, st, nullptr));
    for (int64_t c = 0; c + gw < n; c += gw) {
        // the group at c is factored and its copies are in buffer cur; the
        // joint update covers rows and columns [c2, n), c2 = c + G nb, the
        // next group, whose panel 0 is at index i2 = c2 - b0
        const int64_t b0 = c + nb, c2 = c + gw, i2 = c2 - b0, m2 = n - c2;
        const int64_t w0 = m2 < nb ? m2 : nb;
        if (!la) {
            HPLX_PROPAGATE(update(b0, cur, i2, m2, i2, m2, gw, st));
            HPLX_PROPAGATE(fact(c2, w0, st));
            if (m2 > w0) HPLX_PROPAGATE(group_panels(c2, cur ^ 1, st, nullptr));
        } else {
            hipEvent_t *ev = d->ev_mxp;
            int64_t done = i2;  // rows and columns [b0 + done, n) still to update: the rest
            for (int64_t i = 0; i < G && done < n - b0; ++i) {
                const int64_t wi = (n - b0 - done) < nb ? (n - b0 - done) : nb;
                HPLX_PROPAGATE(update(b0, cur, done, n - b0 - done, done, wi, gw, st));  // panel i's columns
                HPLX_TRY(hipEventRecord(ev[2 * i], st));
                if (i == 0) {
                    HPLX_TRY(hipStreamWaitEvent(sp, ev[0], 0));
                    HPLX_PROPAGATE(fact(c2, w0, sp));
                }
                HPLX_PROPAGATE(update(b0, cur, done, wi, done + wi, n - b0 - done - wi, gw, st));  // its rows
                HPLX_TRY(hipEventRecord(ev[2 * i + 1], st));
                done += wi;
            }
            if (m2 > w0) HPLX_PROPAGATE(group_panels(c2, cur ^ 1, sp, ev));
            HPLX_PROPAGATE(update(b0, cur, done, n - b0 - done, done, n - b0 - done, gw, st));  // the rest
            HPLX_TRY(hipEventRecord(ev[2 * kMxpMaxGroup], sp));
            HPLX_TRY(hipStreamWaitEvent(st, ev[2 * kMxpMaxGroup], 0));
        }
        cur ^= 1;
    }
    unsigned long long hinfo = 0;
    HPLX_TRY(hipMemcpyAsync(&hinfo, dinfo, sizeof hinfo, hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    HPLX_PROPAGATE(tm.collect());
    *info = (hinfo == ULLONG_MAX) ? 0 : (int64_t)hinfo;
    return HPL_OK;
}

static int mxp_solve_impl(Device *d, const double *A, int64_t lda, const float *LU, int64_t ldlu, int64_t n,
                          const double *b, double *x, int64_t max_iter, double *out, hipStream_t st)
{
    const int64_t need = (2 + 2 * (int64_t)kResSplit) * n;  // r, d, partial sums
    if (d->mxp_vec_cap < need) {
        if (d->mxp_vec) HPLX_TRY(hipFree(d->mxp_vec));
        d->mxp_vec = nullptr;
        d->mxp_vec_cap = 0;
        if (hipMalloc((void **)&d->mxp_vec, sizeof(double) * (size_t)need) != hipSuccess)
            HPLX_FAIL(HPL_ERR_NOMEM, "refinement vectors allocation failed");
        d->mxp_vec_cap = need;
    }
    HPLX_PROPAGATE(ensure_red(d, 4));
    double *r = d->mxp_vec, *dv = d->mxp_vec + n, *part = d->mxp_vec + 2 * n;
    const int64_t bs = 64;
    const int64_t nblk = (n + bs - 1) / bs;
    auto lu_solve = [&](double *v) -> int {  // v <- U^{-1} L^{-1} v with the FP32 factors
        for (int64_t q = 0; q < nblk; ++q) {
            const int64_t r0 = q * bs, bb = (n - r0) < bs ? (n - r0) : bs;
            HPLX_PROPAGATE(launch_solve_block_f32(LU, ldlu, v, n, 1, r0, bb, r0 + bb, n, 0, d->solve_done, st));
        }
        for (int64_t q = nblk - 1; q >= 0; --q) {
            const int64_t r0 = q * bs, bb = (n - r0) < bs ? (n - r0) : bs;
            HPLX_PROPAGATE(launch_solve_block_f32(LU, ldlu, v, n, 1, r0, bb, 0, r0, 1, d->solve_done, st));
        }
        return HPL_OK;
    };
    HPLX_TRY(hipMemcpyAsync(x, b, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
    HPLX_PROPAGATE(lu_solve(x));
    const double eps = 0x1.0p-53;
    double anorm = 0.0, scaled = 0.0, rn = 0.0, xn = 0.0, bn = 0.0;
    int64_t it = 0;
    for (;;) {
        HPLX_PROPAGATE(launch_fill_u64(d->red, 4, 0ull, st));
        HPLX_PROPAGATE(launch_mxp_residual(A, lda, x, b, r, n, it == 0, part, d->red, st));
        unsigned long long h[4];
        HPLX_TRY(hipMemcpyAsync(h, d->red, sizeof h, hipMemcpyDeviceToHost, st));
        HPLX_TRY(hipStreamSynchronize(st));
        double v[4];
        memcpy(v, h, sizeof v);
        rn = v[0];
        xn = v[1];
        bn = v[2];
        if (it == 0) anorm = v[3];
        const double den = eps * (anorm * xn + bn) * (double)n;
        scaled = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
        if (!(scaled >= 16.0) || it >= max_iter) break;  // NaN also stops
        HPLX_TRY(hipMemcpyAsync(dv, r, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
        HPLX_PROPAGATE(lu_solve(dv));
        HPLX_PROPAGATE(launch_axpy(x, dv, n, st));
        ++it;
    }
    out[0] = (double)it;
    out[1] = scaled;
    out[2] = rn;
    out[3] = anorm;
    out[4] = xn;
    return HPL_OK;
}

static int residual_impl(const double *A, int64_t lda, bool gen, uint64_t seed, int64_t n, const double *X,
                         int64_t ldx, const double *B, int64_t ldb, int64_t nrhs, double *out, hipStream_t st)
{
    for (int i = 0; i < 5; ++i) out[i] = 0.0;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    const int64_t cnt = 1 + 3 * nrhs;
    HPLX_PROPAGATE(ensure_red(d, cnt));
    HPLX_PROPAGATE(launch_fill_u64(d->red, cnt, 0ull, st));
    HPLX_PROPAGATE(launch_residual(A, lda, gen, gen ? stream_state(seed, 0) : 0, n, X, ldx, B, ldb, nrhs, d->red, st));
    std::vector<unsigned long long> h(cnt);
    HPLX_TRY(hipMemcpyAsync(h.data(), d->red, sizeof(unsigned long long) * cnt, hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    auto asd = [](unsigned long long u) {
        double v;
        memcpy(&v, &u, sizeof v);
        return v;
    };
    const double eps = 0x1.0p-53;
    const double anorm = asd(h[0]);
    double worst = 0.0, rmax = 0.0, xmax = 0.0, bmax = 0.0;
    auto upd = [](double &acc, double v) {
        if (!(v <= acc)) acc = v;  // NaN wins
    };
    for (int64_t c = 0; c < nrhs; ++c) {
        const double rn = asd(h[1 + 3 * c]), xn = asd(h[2 + 3 * c]), bn = asd(h[3 + 3 * c]);
        upd(worst, rn / (eps * (anorm * xn + bn) * (double)n));
        upd(rmax, rn);
        upd(xmax, xn);
        upd(bmax, bn);
    }
    out[0] = worst;
    out[1] = rmax;
    out[2] = anorm;
    out[3] = xmax;
    out[4] = bmax;
    return HPL_OK;
}

}  // namespace hplx

using namespace hplx;

extern "C" {

int hpl_factor(double *A, int64_t n, int64_t lda, int64_t nb, int32_t *ipiv, int64_t *info, void *hip_stream)
{
    if (n > 0 && A == nullptr) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (nb < 1 || nb > (int64_t)kMaxChunks * kMaxSwaps) return -4;
    if (n > 0 && ipiv == nullptr) return -5;
    if (info == nullptr) return -6;
    *info = 0;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    return factor_impl(d, A, n, lda, nb, ipiv, info, (hipStream_t)hip_stream);
}

int hpl_solve(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n, int64_t lda, int64_t ldb,
              int trans, void *hip_stream)
{
    if (n > 0 && LU == nullptr) return -1;
    if (n > 0 && ipiv == nullptr) return -2;
    if (n > 0 && nrhs > 0 && B == nullptr) return -3;
    if (nrhs < 0) return -4;
    if (n < 0 || n > INT32_MAX) return -5;
    if (lda < (n > 1 ? n : 1)) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (trans != 0 && trans != 1) return -8;
    if (n == 0 || nrhs == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    return solve_impl(d, LU, ipiv, B, nrhs, n, lda, ldb, trans, (hipStream_t)hip_stream);
}

int hpl_solve_augmented(double *A, int64_t n, int64_t lda, int64_t nb, int64_t nrhs, int32_t *ipiv, int64_t *info,
                        void *hip_stream)
{
    if (n > 0 && A == nullptr) return -1;
    if (n < 0 || n > INT32_MAX) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (nb < 1 || nb > (int64_t)kMaxChunks * kMaxSwaps) return -4;
    if (nrhs < 0) return -5;
    if (n > 0 && ipiv == nullptr) return -6;
    if (info == nullptr) return -7;
    *info = 0;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    HPLX_PROPAGATE(factor_impl(d, A, n, lda, nb, ipiv, info, st, nrhs, false));
    if (*info != 0 || nrhs == 0) return HPL_OK;
    // back substitution U X = L^{-1} P^{-1} B on the carried columns
    Timer tm(d, opt_timing.load() != 0);
    int id = tm.begin(ST_SOLVE, st);
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)d->solve_done, 1, 0ull, st));
    HPLX_PROPAGATE(solve_upper_sequence(A, A + off(0, n, lda), nrhs, n, lda, lda, d->solve_done, st));
    HPLX_PROPAGATE(tm.end(id, st, (double)n * (double)n * (double)nrhs, 8.0 * 0.5 * (double)n * (double)n));
    HPLX_TRY(hipStreamSynchronize(st));
    return tm.collect();
}

int hpl_residual(const double *A0, int64_t n, int64_t lda, const double *X, int64_t ldx, const double *B, int64_t ldb,
                 int64_t nrhs, double *out, void *hip_stream)
{
    if (n > 0 && A0 == nullptr) return -1;
    if (n < 0) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (n > 0 && X == nullptr) return -4;
    if (ldx < (n > 1 ? n : 1)) return -5;
    if (n > 0 && B == nullptr) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (nrhs < 1) return -8;
    if (out == nullptr) return -9;
    return residual_impl(A0, lda, false, 0, n, X, ldx, B, ldb, nrhs, out, (hipStream_t)hip_stream);
}

int hpl_residual_gen(uint64_t seed, int64_t n, const double *X, int64_t ldx, const double *B, int64_t ldb,
                     int64_t nrhs, double *out, void *hip_stream)
{
    if (n < 0) return -2;
    if (n > 0 && X == nullptr) return -3;
    if (ldx < (n > 1 ? n : 1)) return -4;
    if (n > 0 && B == nullptr) return -5;
    if (ldb < (n > 1 ? n : 1)) return -6;
    if (nrhs < 1) return -7;
    if (out == nullptr) return -8;
    return residual_impl(nullptr, 1, true, seed, n, X, ldx, B, ldb, nrhs, out, (hipStream_t)hip_stream);
}

int hpl_generate(uint64_t seed, uint64_t stream_id, double *M, int64_t rows, int64_t cols, int64_t ld,
                 void *hip_stream)
{
    if (rows > 0 && cols > 0 && M == nullptr) return -3;
    if (rows < 0) return -4;
    if (cols < 0) return -5;
    if (ld < (rows > 1 ? rows : 1)) return -6;
    if (rows == 0 || cols == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    HPLX_PROPAGATE(launch_generate(stream_state(seed, stream_id), M, rows, cols, ld, st));
    HPLX_TRY(hipStreamSynchronize(st));
    return HPL_OK;
}

int hpl_generate_normal(uint64_t seed, uint64_t stream_id, double *M, int64_t rows, int64_t cols, int64_t ld,
                        void *hip_stream)
{
    if (rows > 0 && cols > 0 && M == nullptr) return -3;
    if (rows < 0) return -4;
    if (cols < 0) return -5;
    if (ld < (rows > 1 ? rows : 1)) return -6;
    if (rows == 0 || cols == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    HPLX_PROPAGATE(launch_generate_normal(stream_state(seed, stream_id), M, rows, cols, ld, st));
    HPLX_TRY(hipStreamSynchronize(st));
    return HPL_OK;
}

int hpl_add_diagonal(double *M, int64_t n, int64_t ld, double alpha, void *hip_stream)
{
    if (n > 0 && M == nullptr) return -1;
    if (n < 0) return -2;
    if (ld < (n > 1 ? n : 1)) return -3;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    HPLX_PROPAGATE(launch_add_diagonal(M, n, ld, alpha, st));
    HPLX_TRY(hipStreamSynchronize(st));
    return HPL_OK;
}

int hpl_solve_grad_a(const double *GB, int64_t ldgb, const double *X, int64_t ldx, int64_t n, int64_t nrhs,
                     double *dA, int64_t ldda, void *hip_stream)
{
    if (n > 0 && nrhs > 0 && GB == nullptr) return -1;
    if (ldgb < (n > 1 ? n : 1)) return -2;
    if (n > 0 && nrhs > 0 && X == nullptr) return -3;
    if (ldx < (n > 1 ? n : 1)) return -4;
    if (n < 0 || n > ((int64_t)65535 * 32)) return -5;
    if (nrhs < 0) return -6;
    if (n > 0 && dA == nullptr) return -7;
    if (ldda < (n > 1 ? n : 1)) return -8;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    Timer tm(d, opt_timing.load() != 0);
    const int id = tm.begin(ST_GRAD_A, st);
    HPLX_PROPAGATE(launch_grad_a(GB, ldgb, X, ldx, n, nrhs, dA, ldda, st));
    HPLX_PROPAGATE(tm.end(id, st, 2.0 * (double)n * (double)n * (double)nrhs,
                          8.0 * (double)n * (double)n + 16.0 * (double)n * (double)nrhs));
    HPLX_TRY(hipStreamSynchronize(st));
    return tm.collect();
}

int hpl_mxp_generate(uint64_t seed, double *A, int64_t n, int64_t lda, void *hip_stream)
{
    if (n > 0 && A == nullptr) return -2;
    if (n < 0) return -3;
    if (lda < (n > 1 ? n : 1)) return -4;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    HPLX_PROPAGATE(launch_generate(stream_state(seed, 0), A, n, n, lda, st));
    HPLX_PROPAGATE(launch_mxp_diag(A, n, lda, st));
    HPLX_TRY(hipStreamSynchronize(st));
    return HPL_OK;
}

int hpl_mxp_factor(const double *A, int64_t n, int64_t lda, int64_t nb, int fmt, float *LU, int64_t ldlu,
                   int64_t *info, void *hip_stream)
{
    if (n > 0 && A == nullptr) return -1;
    if (n < 0 || n > 0x7fffffffll) return -2;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (nb < 64 || nb > 4096 || nb % 64 != 0) return -4;
    if (fmt != 0 && fmt != 1) return -5;
    if (n > 0 && LU == nullptr) return -6;
    if (ldlu < (n > 1 ? n : 1)) return -7;
    if (info == nullptr) return -8;
    *info = 0;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    return mxp_factor_impl(d, A, n, lda, nb, fmt, LU, ldlu, info, (hipStream_t)hip_stream);
}

int hpl_mxp_solve(const double *A, int64_t lda, const float *LU, int64_t ldlu, int64_t n, const double *b, double *x,
                  int64_t max_iter, double *out, void *hip_stream)
{
    if (n > 0 && A == nullptr) return -1;
    if (lda < (n > 1 ? n : 1)) return -2;
    if (n > 0 && LU == nullptr) return -3;
    if (ldlu < (n > 1 ? n : 1)) return -4;
    if (n < 0) return -5;
    if (n > 0 && b == nullptr) return -6;
    if (n > 0 && x == nullptr) return -7;
    if (max_iter < 0) return -8;
    if (out == nullptr) return -9;
    for (int i = 0; i < 5; ++i) out[i] = 0.0;
    if (n == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    return mxp_solve_impl(d, A, lda, LU, ldlu, n, b, x, max_iter, out, (hipStream_t)hip_stream);
}

int hpl_set_option(int key, int64_t value)
{
    switch (key) {
    case HPL_OPT_LOOKAHEAD:
        if (value < 0 || value > 3) return -2;
        opt_lookahead = value;
        return 0;
    case HPL_OPT_PANEL_BASE:
        if (value != 8 && value != 16 && value != 32 && value != 64) return -2;
        opt_panel_base = value;
        return 0;
    case HPL_OPT_PANEL_WGS:
        if (value < 1 || value > kLeafMaxWGs) return -2;
        opt_panel_wgs = value;
        return 0;
    case HPL_OPT_TIMING:
        if (value != 0 && value != 1) return -2;
        opt_timing = value;
        return 0;
    case HPL_OPT_PROGRESS:
        if (value < 0) return -2;
        opt_progress = value;
        return 0;
    case HPL_OPT_SERIALIZE:
        if (value != 0 && value != 1) return -2;
        opt_serialize = value;
        return 0;
    case HPL_OPT_GEMM_TILE:
        if (value < 0 || value > 6) return -2;
        opt_gemm_tile = value;
        return 0;
    case HPL_OPT_HOST_PANEL:
        if (value < 0 || value > kHostPanelMaxThreads) return -2;
        opt_host_panel = value;
        return 0;
    case HPL_OPT_LASWP_WGS:
        if (value < 0 || value > 65536) return -2;
        opt_laswp_wgs = value;
        return 0;
    case HPL_OPT_BATCH_CONFIG:
        if (value < 0 || value > 2 * HPL_BATCH_VARIANTS) return -2;
        opt_batch_config = value;
        return 0;
    default: return -1;
    }
}

int64_t hpl_get_option(int key)
{
    switch (key) {
    case HPL_OPT_LOOKAHEAD: return opt_lookahead;
    case HPL_OPT_PANEL_BASE: return opt_panel_base;
    case HPL_OPT_PANEL_WGS: return opt_panel_wgs;
    case HPL_OPT_TIMING: return opt_timing;
    case HPL_OPT_PROGRESS: return opt_progress;
    case HPL_OPT_SERIALIZE: return opt_serialize;
    case HPL_OPT_GEMM_TILE: return opt_gemm_tile;
    case HPL_OPT_HOST_PANEL: return opt_host_panel;
    case HPL_OPT_LASWP_WGS: return opt_laswp_wgs;
    case HPL_OPT_BATCH_CONFIG: return opt_batch_config;
    default: return INT64_MIN;
    }
}

int hpl_get_stats(int64_t *launches, double *ms, double *flops, double *bytes, int cap)
{
    std::lock_guard<std::mutex> lk(g_st_mu);
    for (int k = 0; k < ST_N && k < cap; ++k) {
        if (launches) launches[k] = g_st_launch[k];
        if (ms) ms[k] = g_st_ms[k];
        if (flops) flops[k] = g_st_flops[k];
        if (bytes) bytes[k] = g_st_bytes[k];
    }
    return ST_N;
}

void hpl_reset_stats(void)
{
    std::lock_guard<std::mutex> lk(g_st_mu);
    for (int k = 0; k < ST_N; ++k) {
        g_st_launch[k] = 0;
        g_st_ms[k] = g_st_flops[k] = g_st_bytes[k] = 0.0;
    }
}

int hpl_mfma_peak(int64_t iters, double *out, void *hip_stream)
{
    if (iters <= 0) return -1;
    if (out == nullptr) return -2;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    int cus = 0;
    HPLX_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->id));
    const int64_t nwg = 2 * (int64_t)cus;  // two 256-thread workgroups per CU
    iters = mfma_peak_rounds(iters);
    HPLX_PROPAGATE(ensure_red(d, nwg * 256));
    double *buf = (double *)d->red;
    // timing events of its own (the device's stream-ordering events carry no timestamps)
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    HPLX_TRY(hipEventCreate(&ev.e0));
    HPLX_TRY(hipEventCreate(&ev.e1));
    HPLX_PROPAGATE(launch_mfma_peak(buf, nwg, mfma_peak_rounds(iters / 16 + 1), st));  // warm-up
    float best = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
        HPLX_TRY(hipEventRecord(ev.e0, st));
        HPLX_PROPAGATE(launch_mfma_peak(buf, nwg, iters, st));
        HPLX_TRY(hipEventRecord(ev.e1, st));
        HPLX_TRY(hipEventSynchronize(ev.e1));
        float ms = 0.0f;
        HPLX_TRY(hipEventElapsedTime(&ms, ev.e0, ev.e1));
        if (rep == 0 || ms < best) best = ms;
    }
    out[0] = best > 0.0f ? mfma_peak_flops(nwg, iters) / ((double)best * 1e-3) / 1e12 : 0.0;
    out[1] = (double)best;
    return HPL_OK;
}

// ---------------------------------------------------------------------------
// batched small systems
// ---------------------------------------------------------------------------
int hpl_batched_sizes(uint64_t seed, int64_t count, int32_t nmin, int32_t nmax, int32_t *sizes)
{
    if (count < 0) return -2;
    if (nmin < 1) return -3;
    if (nmax < nmin) return -4;
    if (count > 0 && sizes == nullptr) return -5;
    const uint64_t s0 = stream_state(seed, kBatchSizeStream);
    const int64_t range = (int64_t)nmax - (int64_t)nmin + 1;
    for (int64_t i = 0; i < count; ++i) {
        const double u = gen_value(s0, (uint64_t)i) + 0.5;  // exact, in [0, 1)
        int64_t k = (int64_t)floor(u * (double)range);
        if (k > range - 1) k = range - 1;
        sizes[i] = (int32_t)(nmin + k);
    }
    return HPL_OK;
}

// The tuned table: kBatchCostUs[occ - 1][variant][bucket], microseconds per
// system amortized over the device, and kBatchTableTuned (0: built-in default).
#include "batched_tuned.inc"
static_assert(sizeof(kBatchCostUs) == sizeof(double) * 2 * HPL_BATCH_VARIANTS * kBatchBuckets, "table shape");
static_assert(kBatchBuckets == HPL_BATCH_BUCKETS, "bucket count");

// Per occ, each bucket's cheapest variant; the occ with the smaller predicted
// sum over the batch wins.
static void batch_choose(int64_t count, const int32_t *sizes, int *occ, signed char *vtab, double *pred_ms)
{
    std::vector<int64_t> hist(kBatchBuckets, 0);
    for (int64_t i = 0; i < count; ++i) ++hist[(size_t)((sizes[i] - 1) >> 5)];
    double best = 1e300;
    for (int o = 0; o < 2; ++o) {
        signed char vt[kBatchBuckets];
        double tot = 0.0;
        for (int q = 0; q < kBatchBuckets; ++q) {
            int bv = 0;
            for (int v = 1; v < HPL_BATCH_VARIANTS; ++v)
                if (kBatchCostUs[o][v][q] < kBatchCostUs[o][bv][q]) bv = v;
            vt[q] = (signed char)bv;
            tot += (double)hist[(size_t)q] * kBatchCostUs[o][bv][q];
        }
        if (tot < best) {
            best = tot;
            *occ = o + 1;
            memcpy(vtab, vt, sizeof vt);
        }
    }
    if (pred_ms) *pred_ms = best * 1e-3;
}

int hpl_batched_config(int64_t count, const int32_t *sizes, int *occ, int8_t *vtab, double *predicted_ms)
{
    if (count < 0) return -1;
    if (count > 0 && sizes == nullptr) return -2;
    for (int64_t i = 0; i < count; ++i)
        if (sizes[i] < 1 || sizes[i] > kBatchMaxN) return -2;
    if (occ == nullptr) return -3;
    if (vtab == nullptr) return -4;
    batch_choose(count, sizes, occ, (signed char *)vtab, predicted_ms);
    return HPL_OK;
}

int hpl_batched_table(double *cost, int *tuned)
{
    if (cost == nullptr) return -1;
    if (tuned == nullptr) return -2;
    for (int o = 0; o < 2; ++o)
        for (int v = 0; v < HPL_BATCH_VARIANTS; ++v)
            for (int q = 0; q < kBatchBuckets; ++q)
                cost[((size_t)o * HPL_BATCH_VARIANTS + v) * kBatchBuckets + q] = kBatchCostUs[o][v][q];
    *tuned = kBatchTableTuned;
    return HPL_OK;
}

int hpl_batched_solve(int64_t count, const int32_t *sizes, int64_t nrhs, double *A, int32_t *ipiv, double *B,
                      const double *W, double *GB, double *GA, int mode, int64_t *info, void *hip_stream)
{
    if (count < 0) return -1;
    if (count > 0 && sizes == nullptr) return -2;
    if (nrhs < 1 || nrhs > kBatchMaxRhs) return -3;
    if (mode < 1 || mode > 3) return -10;
    if (count > 0 && info == nullptr) return -11;
    for (int64_t i = 0; i < count; ++i)
        if (sizes[i] < 1 || sizes[i] > kBatchMaxN) return -2;
    if (count > 0 && (A == nullptr || ipiv == nullptr || B == nullptr)) return A == nullptr ? -4 : (ipiv == nullptr ? -5 : -6);
    if ((mode & 2) && count > 0 && (W == nullptr || GB == nullptr || GA == nullptr))
        return W == nullptr ? -7 : (GB == nullptr ? -8 : -9);
    if (count == 0) return HPL_OK;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    // host plan: packed offsets and the largest-first order
    std::vector<int64_t> aoff((size_t)count), voff((size_t)count);
    std::vector<int32_t> order((size_t)count);
    int64_t a_acc = 0, v_acc = 0;
    for (int64_t i = 0; i < count; ++i) {
        aoff[(size_t)i] = a_acc;
        voff[(size_t)i] = v_acc;
        a_acc += (int64_t)sizes[i] * sizes[i];
        v_acc += sizes[i];
        order[(size_t)i] = (int32_t)i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return sizes[x] > sizes[y]; });
    // device copies: sizes | aoff | voff | order | info | counter (256-byte aligned pieces)
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_sizes = 0, o_aoff = up(4 * (size_t)count), o_voff = o_aoff + up(8 * (size_t)count);
    const size_t o_order = o_voff + up(8 * (size_t)count), o_info = o_order + up(4 * (size_t)count);
    const size_t o_cnt = o_info + up(8 * (size_t)count), total = o_cnt + 256;
    if (d->bat_cap < total) {
        if (d->bat_ws) HPLX_TRY(hipFree(d->bat_ws));
        d->bat_ws = nullptr;
        d->bat_cap = 0;
        if (hipMalloc(&d->bat_ws, total) != hipSuccess) HPLX_FAIL(HPL_ERR_NOMEM, "batched workspace allocation failed");
        d->bat_cap = total;
    }
    char *ws = (char *)d->bat_ws;
    HPLX_TRY(hipMemcpyAsync(ws + o_sizes, sizes, 4 * (size_t)count, hipMemcpyHostToDevice, st));
    HPLX_TRY(hipMemcpyAsync(ws + o_aoff, aoff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, st));
    HPLX_TRY(hipMemcpyAsync(ws + o_voff, voff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, st));
    HPLX_TRY(hipMemcpyAsync(ws + o_order, order.data(), 4 * (size_t)count, hipMemcpyHostToDevice, st));
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)(ws + o_cnt), 1, 0ull, st));
    int cus = 0;
    HPLX_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d->id));
    int occ = 1;
    signed char vtab[kBatchBuckets];
    const int64_t forced = opt_batch_config.load();
    if (forced == 0) {
        batch_choose(count, sizes, &occ, vtab, nullptr);
    } else {
        occ = 1 + (int)((forced - 1) / HPL_BATCH_VARIANTS);
        memset(vtab, (int)((forced - 1) % HPL_BATCH_VARIANTS), sizeof vtab);
    }
    Timer tm(d, opt_timing.load() != 0);
    const int id = tm.begin(ST_BATCHED, st);
    HPLX_PROPAGATE(launch_batched_solve(count, (const int32_t *)(ws + o_sizes), (const int64_t *)(ws + o_aoff),
                                        (const int64_t *)(ws + o_voff), (const int32_t *)(ws + o_order), A, ipiv, B,
                                        W, GB, GA, (int)nrhs, mode, (int64_t *)(ws + o_info),
                                        (unsigned *)(ws + o_cnt), occ, vtab, cus, st));
    double fl = 0.0;
    for (int64_t i = 0; i < count; ++i) {
        const double n = (double)sizes[i];
        if (mode & 1) fl += 2.0 * n * n * n / 3.0 + 2.0 * n * n * (double)nrhs;
        if (mode & 2) fl += 2.0 * n * n * (double)nrhs + 2.0 * n * n * (double)nrhs;
    }
    HPLX_PROPAGATE(tm.end(id, st, fl, 8.0 * (double)a_acc * ((mode & 2) ? 3.0 : 2.0)));
    HPLX_TRY(hipMemcpyAsync(info, ws + o_info, 8 * (size_t)count, hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    return tm.collect();
}

int hpl_host_panel(double *P, int64_t m, int64_t nb, int64_t ldp, int32_t *ipiv, int threads, int64_t *info)
{
    if (m < 0) return -2;
    if (nb < 1 || nb > m) return m == 0 ? (info ? (*info = 0, 0) : -7) : -3;
    if (m > 0 && P == nullptr) return -1;
    if (ldp < (m > 1 ? m : 1)) return -4;
    if (ipiv == nullptr) return -5;
    if (threads < 1 || threads > kHostPanelMaxThreads) return -6;
    if (info == nullptr) return -7;
    return host_panel_factor(P, m, nb, ldp, ipiv, threads, info);
}

int hpl_panel_factor(double *A, int64_t m, int64_t nb, int64_t lda, int32_t *ipiv, int64_t *info, void *hip_stream)
{
    if (m < 0) return -2;
    if (nb < 1 || nb > 1024 || nb > m) return m == 0 ? (info ? (*info = 0, 0) : -6) : -3;
    if (A == nullptr) return -1;
    if (lda < (m > 1 ? m : 1)) return -4;
    if (ipiv == nullptr) return -5;
    if (info == nullptr) return -6;
    Device *d = nullptr;
    HPLX_PROPAGATE(get_device(&d));
    hipStream_t st = (hipStream_t)hip_stream;
    Timer tm(d, opt_timing.load() != 0);
    Ctx x{d, A, m, lda, ipiv, (int)opt_panel_base.load(), (int)opt_panel_wgs.load(), (int)opt_gemm_tile.load(), &tm};
    HPLX_PROPAGATE(launch_fill_u64(d->sync.info, 1, ULLONG_MAX, st));
    HPLX_PROPAGATE(panel_full(x, 0, nb, d->ring[0], st));
    HPLX_TRY(hipMemcpyAsync(d->hbuf, d->sync.info, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipMemcpyAsync(d->hbuf + 1, d->sync.abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    HPLX_PROPAGATE(tm.collect());
    if (*(int *)(d->hbuf + 1)) HPLX_FAIL(HPL_ERR_INTERNAL, "panel barrier timed out");
    const unsigned long long iv = d->hbuf[0];
    *info = (iv == ULLONG_MAX) ? 0 : (int64_t)iv;
    return HPL_OK;
}

int hpl_release(void)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return HPL_OK;
    for (int i = 0; i < kMaxDevices; ++i) {
        Device &d = g_dev[i];
        if (!d.ready) continue;
        HPLX_TRY(hipSetDevice(i));
        HPLX_TRY(hipDeviceSynchronize());
        for (hipEvent_t e : d.ev_pool) (void)hipEventDestroy(e);
        d.ev_pool.clear();
        for (int r = 0; r < kRing; ++r) {
            (void)hipEventDestroy(d.ev_panel[r]);
            (void)hipEventDestroy(d.ev_la[r]);
            (void)hipEventDestroy(d.ev_iter[r]);
        }
        for (hipEvent_t e : d.ev_mxp) (void)hipEventDestroy(e);
        (void)hipEventDestroy(d.ev_start);
        (void)hipEventDestroy(d.ev_end);
        (void)hipStreamDestroy(d.sp);
        if (d.red) (void)hipFree(d.red);
        if (d.splans) (void)hipFree(d.splans);
        if (d.mxp_ws) (void)hipFree(d.mxp_ws);
        if (d.mxp_vec) (void)hipFree(d.mxp_vec);
        if (d.bat_ws) (void)hipFree(d.bat_ws);
        if (d.hp_buf) (void)hipHostFree(d.hp_buf);
        if (d.hbuf) (void)hipHostFree(d.hbuf);
        (void)hipFree(d.ws);
        d = Device();
    }
    HPLX_TRY(hipSetDevice(cur));
    return HPL_OK;
}

const char *hpl_strerror(int code)
{
    static const char *neg[] = {"",
                                "invalid argument 1",
                                "invalid argument 2",
                                "invalid argument 3",
                                "invalid argument 4",
                                "invalid argument 5",
                                "invalid argument 6",
                                "invalid argument 7",
                                "invalid argument 8",
                                "invalid argument 9",
                                "invalid argument 10"};
    switch (code) {
    case HPL_OK: return "success";
    case HPL_ERR_HIP: return "HIP runtime error";
    case HPL_ERR_NOMEM: return "workspace allocation failed";
    case HPL_ERR_DEVICE: return "no gfx950 device";
    case HPL_ERR_INTERNAL: return "internal error (kernel-reported failure)";
    default:
        if (code < 0 && code >= -10) return neg[-code];
        return "unknown error code";
    }
}

const char *hpl_last_error_detail(void)
{
    return g_err_detail;
}

}  // extern "C"
