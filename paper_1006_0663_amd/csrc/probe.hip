// FP64 FMA throughput probe (declared in include/teuk.h): the attainable
// FP64 vector rate of the device, against which the step kernels' FP64
// operation rates are read.  Every lane runs `chains` independent chains
// x <- fma(x, a, b); a launch of `blocks` x `threads` lanes for `iters`
// iterations performs 2 * chains * iters * blocks * threads FP64 operations.
#include "teuk.h"

#include <hip/hip_runtime.h>

#include <string>

namespace {

template <int CH>
__global__ void fma_probe_kernel(double a, double b, long iters, double *out) {
    double x[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) x[c] = 1e-3 * threadIdx.x + c;
    for (long it = 0; it < iters; it += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < CH; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) s += x[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;      // keeps every chain live
}

hipError_t launch_probe(int chains, int blocks, int threads, long iters, double *out, hipStream_t st) {
    // a = 1 - 2^-10, b = 2^-10: every chain converges to 1, no overflow or subnormals
    const double a = 1.0 - 1.0 / 1024.0, b = 1.0 / 1024.0;
    switch (chains) {
        case 1: fma_probe_kernel<1><<<blocks, threads, 0, st>>>(a, b, iters, out); break;
        case 2: fma_probe_kernel<2><<<blocks, threads, 0, st>>>(a, b, iters, out); break;
        case 4: fma_probe_kernel<4><<<blocks, threads, 0, st>>>(a, b, iters, out); break;
        case 8: fma_probe_kernel<8><<<blocks, threads, 0, st>>>(a, b, iters, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" int teuk_fp64_fma_probe(int chains, int blocks, int threads, long iters, double *tflops, double *ms) {
    if ((chains != 1 && chains != 2 && chains != 4 && chains != 8) || blocks < 1 || blocks > (1 << 20) ||
        threads < 64 || threads > 1024 || threads % 64 != 0 || iters < 8 || iters % 8 != 0 || !tflops)
        return TEUK_EINVAL;
    double *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&out, (size_t)blocks * threads * sizeof(double));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_probe(chains, blocks, threads, iters, out, st);     // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_probe(chains, blocks, threads, iters, out, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) {
        *tflops = 2.0 * chains * (double)iters * blocks * threads / (t * 1e-3) / 1e12;
        if (ms) *ms = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(out);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? TEUK_ENOMEM : TEUK_EDEVICE;
    return TEUK_OK;
}
