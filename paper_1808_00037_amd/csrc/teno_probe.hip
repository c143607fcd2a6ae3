// teno_probe.hip -- measurement support: the device's FP64 vector FMA rate, so that the sweeps'
// counted flops can be set against a peak measured on the same device beside the published one.
#include <hip/hip_runtime.h>

#include "teno.h"

namespace {

constexpr int PROBE_CHAINS = 8;       // independent FMA chains per thread (covers the FMA latency)
constexpr int PROBE_BLOCK = 256;

// Each thread runs PROBE_CHAINS dependent FMA chains of `iters` steps in registers; one store per
// thread keeps the work live.
__global__ void __launch_bounds__(PROBE_BLOCK) fma_probe_kernel(int iters, double a, double b, double *out)
{
    double x[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = (double)(threadIdx.x + c) * 1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += x[c];
    out[(size_t)blockIdx.x * PROBE_BLOCK + threadIdx.x] = s;
}

}  // namespace

extern "C" teno_status teno_probe_fp64_fma(void *stream, int32_t iters, double *tflops)
{
    if (!tflops || iters < 1 || iters > (1 << 24)) return TENO_E_ARG;
    *tflops = 0.0;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return TENO_E_HIP;
    const int blocks = ncu * 16;        // several resident blocks per compute unit
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = (hipStream_t)stream;
    teno_status st = TENO_E_HIP;
    if (hipMalloc(&out, (size_t)blocks * PROBE_BLOCK * sizeof(double)) == hipSuccess &&
        hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        float ms = 0.f;
        hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(PROBE_BLOCK), 0, s, 16, 0.999, 1e-3, out);  // warm-up
        (void)hipEventRecord(e0, s);
        hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(PROBE_BLOCK), 0, s, iters, 0.999, 1e-3, out);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f) {
            const double flops = 2.0 * PROBE_CHAINS * (double)iters * (double)blocks * PROBE_BLOCK;
            *tflops = flops / (ms * 1e-3) / 1e12;
            st = TENO_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return st;
}
