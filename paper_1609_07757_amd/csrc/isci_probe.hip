// Measurement aids, not part of the method: FP64 issue-rate probes used to
// re-measure the chip's peaks next to the published figures.  Each kernel
// runs chains of independent FP64 operations on register operands and
// writes one value per thread (so the work is not removed).
#include <hip/hip_runtime.h>

#include "isci_internal.h"

namespace isci {

typedef double v4d_pr __attribute__((ext_vector_type(4)));

// eight independent 16x16x4 FP64 MFMA chains per wave, advanced 16 times
// per step: 16 x 8 x 2048 flops per step and wave.  The step is unrolled so
// that any copy of the accumulators the compiler places at the loop edge is
// paid once per 128 products, not once per 8.
constexpr int kProbeMfmaUnroll = 16;

__global__ __launch_bounds__(256) void k_probe_mfma(int64_t iters, double *__restrict__ out)
{
    v4d_pr acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = v4d_pr{0.0, 0.0, 0.0, 0.0};
    const double a = 1e-9 * (threadIdx.x + 1), b = 1e-9 * (blockIdx.x + 1);
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
        for (int r = 0; r < kProbeMfmaUnroll; ++r)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// sixteen independent FP64 FMA chains per lane: 16 x 2 flops per step
__global__ __launch_bounds__(256) void k_probe_fma(int64_t iters, double *__restrict__ out)
{
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 1e-3 * q;
    const double a = 1.0 - 1e-12 * threadIdx.x, b = 1e-9 * (blockIdx.x + 1);
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = fma(acc[q], a, b);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += acc[q];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace isci

using namespace isci;

extern "C" {

isci_status isci_probe_fp64(int kind, int64_t iters, int blocks, double *out, double *flops, hipStream_t stream)
{
    if (!out || !flops || iters < 1 || blocks < 1 || (kind != 0 && kind != 1)) {
        set_error("isci_probe_fp64: bad argument");
        return ISCI_E_INVALID;
    }
    if (kind == 0) {
        k_probe_mfma<<<blocks, 256, 0, stream>>>(iters, out);
        *flops = (double)blocks * 4.0 * (double)iters * kProbeMfmaUnroll * 8.0 * 2048.0;   // 4 waves per block
    } else {
        k_probe_fma<<<blocks, 256, 0, stream>>>(iters, out);
        *flops = (double)blocks * 256.0 * (double)iters * 16.0 * 2.0;
    }
    ISCI_HIP(hipGetLastError());
    return ISCI_OK;
}

}  // extern "C"
