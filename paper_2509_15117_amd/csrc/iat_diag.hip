// Diagnostics: the FP64 vector rate this GPU sustains on dense independent FMAs, the denominator
// that the achieved FLOP rates of the integrator are compared with next to the published peak.
#include <hip/hip_runtime.h>

#include "iat_host.h"

namespace iat {

// Eight independent FMA chains per lane; every lane writes one value so nothing is dead code.
__global__ void __launch_bounds__(256) k_fma_peak(double* out, int iters, double a, double b)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x0 = 1e-3 * (t & 15), x1 = x0 + 1.0, x2 = x0 + 2.0, x3 = x0 + 3.0;
    double x4 = x0 + 4.0, x5 = x0 + 5.0, x6 = x0 + 6.0, x7 = x0 + 7.0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x0 = fma(x0, a, b);
            x1 = fma(x1, a, b);
            x2 = fma(x2, a, b);
            x3 = fma(x3, a, b);
            x4 = fma(x4, a, b);
            x5 = fma(x5, a, b);
            x6 = fma(x6, a, b);
            x7 = fma(x7, a, b);
        }
    }
    out[t] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

}  // namespace iat

using namespace iat;

extern "C" int iat_fp64_peak(double* scratch, int64_t n_threads, int iters, double* tflops, void* stream)
{
    if (!scratch || !tflops || n_threads < 256 || n_threads % 256 != 0 || iters < 1)
        return set_error(IAT_EINVAL, "fp64_peak: scratch, tflops, n_threads (a multiple of 256) and iters required");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(IAT_EHIP, "hipEventCreate failed");
    const dim3 grid((unsigned)(n_threads / 256));
    hipLaunchKernelGGL(k_fma_peak, grid, dim3(256), 0, st, scratch, 8, 0.999999, 1e-9);   // warm-up
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_fma_peak, grid, dim3(256), 0, st, scratch, iters, 0.999999, 1e-9);
    (void)hipEventRecord(e1, st);
    int rc = 0;
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = set_error(IAT_EHIP, "fp64_peak: timing failed");
    else
        *tflops = 2.0 * 64.0 * (double)iters * (double)n_threads / (ms * 1e-3) / 1e12;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
