// noalloc.hip -- hpl_solve_noalloc: the solve of hpl_solve (same kernels, same
// launch sequence, so the same bits) for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// hpl_solve keeps its scratch (the interchange plans of every 512-pivot chunk
// of ipiv, the workgroup counter of the block launches and the pivot-error
// word) in library workspace that it allocates on first use.  Here that
// scratch is a file-scope device array of fixed size, which every GPU the
// library runs on holds until the process ends.  Its device address is taken
// once per device with hipGetSymbolAddress (the array's name is only a host
// stand-in and is never passed to a kernel or a copy); after that no call
// allocates anything: no hipMalloc, no events, no library workspace.
//
// All calls on one GPU share that GPU's array, so calls that overlap in time
// on one GPU (on different streams, or from different host threads) race.
// Every call clears the words that must start at zero (counter, error word)
// with a fill kernel before using them.
#include "common.hpp"

#include <cstring>
#include <mutex>

namespace hplx {

namespace {

constexpr int64_t kNoAllocMaxN = HPL_SOLVE_NOALLOC_MAX_N;
constexpr int64_t kNoAllocChunks = (kNoAllocMaxN + kMaxSwaps - 1) / kMaxSwaps;
constexpr size_t kOffDone = 0;    // unsigned: workgroup counter of the block launches
constexpr size_t kOffErr = 256;   // int: raised by the plan kernel on a pivot outside [k, n)
constexpr size_t kOffPlans = 512; // int32 plans, kPlanStride per chunk
constexpr size_t kScratchBytes = kOffPlans + sizeof(int32_t) * (size_t)kPlanStride * (size_t)kNoAllocChunks;
static_assert(kScratchBytes == HPL_SOLVE_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDev = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[kMaxDev] = {};  // device address of `scratch` on each device (null: not set up)

// Set-up, once per device with that device current: the architecture check and
// the device address of the scratch array.
int noalloc_scratch(unsigned char **out)
{
    int id = 0;
    HPLX_TRY(hipGetDevice(&id));
    if (id < 0 || id >= kMaxDev) {
        note_error("device index out of range", __FILE__, __LINE__);
        return HPL_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (g_na_ptr[id] == nullptr) {
        hipDeviceProp_t prop;
        HPLX_TRY(hipGetDeviceProperties(&prop, id));
        if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            note_error("device is not gfx950", __FILE__, __LINE__);
            return HPL_ERR_DEVICE;
        }
        void *p = nullptr;
        HPLX_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (p == nullptr) {
            note_error("hipGetSymbolAddress returned no address for the scratch array", __FILE__, __LINE__);
            return HPL_ERR_INTERNAL;
        }
        g_na_ptr[id] = (unsigned char *)p;
    }
    *out = g_na_ptr[id];
    return HPL_OK;
}

}  // namespace

}  // namespace hplx

using namespace hplx;

extern "C" int hpl_solve_noalloc(const double *LU, const int32_t *ipiv, double *B, int64_t nrhs, int64_t n,
                                 int64_t lda, int64_t ldb, int trans, void *hip_stream)
{
    if (n > 0 && LU == nullptr) return -1;
    if (n > 0 && ipiv == nullptr) return -2;
    if (n > 0 && nrhs > 0 && B == nullptr) return -3;
    if (nrhs < 0) return -4;
    if (n < 0) return -5;
    if (n > kNoAllocMaxN) {
        note_error("n exceeds HPL_SOLVE_NOALLOC_MAX_N, the size the fixed scratch array holds plans for",
                   __FILE__, __LINE__);
        return -5;
    }
    if (lda < (n > 1 ? n : 1)) return -6;
    if (ldb < (n > 1 ? n : 1)) return -7;
    if (trans != 0 && trans != 1) return -8;
    if (n == 0 || nrhs == 0) return HPL_OK;
    unsigned char *s = nullptr;
    HPLX_PROPAGATE(noalloc_scratch(&s));
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned *done = (unsigned *)(s + kOffDone);
    int *perr = (int *)(s + kOffErr);
    int32_t *plans = (int32_t *)(s + kOffPlans);
    // the counter and the error word start at zero (a fill kernel: no memset node)
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)done, 1, 0ull, st));
    HPLX_PROPAGATE(launch_fill_u64((unsigned long long *)perr, 1, 0ull, st));
    HPLX_PROPAGATE(solve_sequence(LU, ipiv, B, nrhs, n, lda, ldb, trans, plans, perr, done, st));
    int err = 0;
    HPLX_TRY(hipMemcpyAsync(&err, perr, sizeof(int), hipMemcpyDeviceToHost, st));
    HPLX_TRY(hipStreamSynchronize(st));
    if (err != 0) {
        note_error("pivot index outside [k, n) in ipiv", __FILE__, __LINE__);
        return HPL_ERR_INTERNAL;
    }
    return HPL_OK;
}
