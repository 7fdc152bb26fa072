// Measurement support of the library: the attainable FP64 vector rate (a
// pure fused-multiply-add kernel), which the benchmark's rooflines quote
// beside the chip's published peak.

#include "hydro_common.h"

namespace {

// Attainable FP64 vector rate: each thread runs eight independent chains of
// a = a * m + c (fused multiply-adds, two flops each), iters times, and
// writes their sum; with m = 1 and c = 1 chain k of thread t ends at
// t + k + iters exactly.
__global__ void __launch_bounds__(256) fp64_fma_probe(double *out, int iters, double m, double c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (double)(t + k);
#pragma unroll 1
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = fma(a[k], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    out[t] = s;
}

}  // namespace

hipError_t hydro_launch_fp64_probe(double *out, int blocks, int iters, double m, double c, hipStream_t s) {
    hipLaunchKernelGGL(fp64_fma_probe, dim3(blocks), dim3(256), 0, s, out, iters, m, c);
    return hipGetLastError();
}
