// probe.hip -- measured FP64 matrix-core peak of the device.
//
// A pure v_mfma_f64_16x16x4_f64 issue loop: every wave keeps 16 independent
// accumulator blocks (in AGPRs, the form the GEMM uses) and issues the MFMAs
// back to back, two 256-thread workgroups per CU.  The operands are fixed
// register values, so the loop measures instruction throughput and the clock
// the chip holds while doing nothing else; the sum of the accumulators is
// written out so that no MFMA is dead code.
#include "common.hpp"

namespace hplx {

namespace {

constexpr int kPeakChains = 16;
constexpr int kPeakUnroll = 8;

__global__ __launch_bounds__(256, 2) void mfma_peak_kernel(double *__restrict__ out, int64_t iters, double a,
                                                           double b)
{
    asm volatile("" ::: "a0");  // accumulators in AGPRs
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = (d4){0.0, 0.0, 0.0, 0.0};
    const double av = a + 1e-3 * (double)(threadIdx.x & 63);
    const double bv = b - 1e-3 * (double)(threadIdx.x & 63);
    // kPeakUnroll rounds per loop trip: the compiler copies loop-carried
    // accumulator tuples at the back edge, which would otherwise cost as much
    // as the MFMAs themselves
    for (int64_t it = 0; it < iters; it += kPeakUnroll) {
#pragma unroll
        for (int u = 0; u < kPeakUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kPeakChains; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

int launch_mfma_peak(double *out, int64_t nwg, int64_t iters, hipStream_t st)
{
    if (nwg <= 0 || nwg > 0x7fffffffll || iters <= 0 || iters % kPeakUnroll) return HPL_ERR_INTERNAL;
    hipLaunchKernelGGL(mfma_peak_kernel, dim3((unsigned)nwg), dim3(256), 0, st, out, iters, 0.5, 0.25);
    HPLX_TRY_LAUNCH();
    return HPL_OK;
}

int64_t mfma_peak_rounds(int64_t iters)
{
    return (iters + kPeakUnroll - 1) / kPeakUnroll * kPeakUnroll;
}

double mfma_peak_flops(int64_t nwg, int64_t iters)
{
    // per MFMA: 16 x 16 x 4 multiply-adds
    return (double)nwg * 4.0 * (double)iters * (double)kPeakChains * 2.0 * 16.0 * 16.0 * 4.0;
}

}  // namespace hplx
