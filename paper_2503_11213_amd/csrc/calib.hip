// Roofline calibration: a kernel of known float64 FMA count, so that the
// profiler's float64 FLOP and VALU counters can be scaled before they are
// read on the trace (whose FLOPs are counted from its algorithm).  Not part
// of the method: measurement infrastructure only.
#include <hip/hip_runtime.h>

#include "../../include/sdirt.h"

namespace sdirt {

constexpr int kCalibBlock = 256;
constexpr int kCalibChains = 8;

// Every thread runs kCalibChains independent chains of `iters` dependent
// v_fma_f64 each: exactly n_threads * iters * kCalibChains FMAs
// (2 FLOPs each), and one store per thread so the chains stay live.
__global__ __launch_bounds__(kCalibBlock) void calib_fma64_kernel(long long n_threads,
                                                                  int iters, double* out) {
    const long long t = (long long)blockIdx.x * kCalibBlock + threadIdx.x;
    if (t >= n_threads) return;
    double a[kCalibChains];
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) a[c] = 1e-3 * (double)(t + c);
    const double m = 0.999999, k = 1e-9;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kCalibChains; ++c) a[c] = fma(a[c], m, k);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kCalibChains; ++c) s += a[c];
    out[t] = s;
}

int calib_fma64(long long n_threads, int iters, double* out, hipStream_t st) {
    if (!out || n_threads < 1 || iters < 1) return SDIRT_EINVAL;
    const long long blocks = (n_threads + kCalibBlock - 1) / kCalibBlock;
    if (blocks > 0x7fffffffLL) return SDIRT_EUNSUPPORTED;
    hipLaunchKernelGGL(calib_fma64_kernel, dim3((unsigned)blocks), dim3(kCalibBlock), 0, st,
                       n_threads, iters, out);
    return hipGetLastError() == hipSuccess ? SDIRT_OK : SDIRT_ELAUNCH;
}

}  // namespace sdirt
