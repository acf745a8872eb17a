// Test hooks exposing single multiword operations (include/teuk.h:
// teuk_arith_host / teuk_arith_device) so that the arithmetic can be checked
// against an independent high-precision library, on the CPU and on the GPU.
#include "teuk.h"

#include <hip/hip_runtime.h>

#include <vector>

#include "kernels.hpp"

namespace lwk {

template <class T> MPA T arith_op(int op, T a, T b) {
    T s, c;
    switch (op) {
        case 0: return mp_add(a, b);
        case 1: return mp_sub(a, b);
        case 2: return mp_mul(a, b);
        case 3: return mp_mul_d(a, mp_lead(b));
        case 4: return mp_div(a, b);
        case 5: return mp_sqrt(a);
        case 6: return mp_exp(a);
        case 7: return mp_log(a);
        case 8: mp_sincos(a, s, c); return s;
        default: mp_sincos(a, s, c); return c;
    }
}

template <class T> __global__ void arith_kernel(int op, const double *a, const double *b, double *out, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    constexpr int W = words_of<T>::value;
    const T r = arith_op<T>(op, from_words<T>(a + (size_t)k * W), from_words<T>(b + (size_t)k * W));
    for (int w = 0; w < W; ++w) out[(size_t)k * W + w] = mp_word(r, w);
}

template <class T> void arith_host(int op, const double *a, const double *b, double *out, int n) {
    constexpr int W = words_of<T>::value;
    for (int k = 0; k < n; ++k) {
        const T r = arith_op<T>(op, from_words<T>(a + (size_t)k * W), from_words<T>(b + (size_t)k * W));
        for (int w = 0; w < W; ++w) out[(size_t)k * W + w] = mp_word(r, w);
    }
}

template <class T> int arith_device(int op, const double *a, const double *b, double *out, int n) {
    constexpr int W = words_of<T>::value;
    const size_t bytes = (size_t)n * W * sizeof(double);
    double *d = nullptr;
    if (hipMalloc((void **)&d, 3 * bytes) != hipSuccess) return TEUK_ENOMEM;
    hipError_t e = hipMemcpy(d, a, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + (size_t)n * W, b, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        arith_kernel<T><<<(n + 127) / 128, 128>>>(op, d, d + (size_t)n * W, d + 2 * (size_t)n * W, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, d + 2 * (size_t)n * W, bytes, hipMemcpyDeviceToHost);
    hipFree(d);
    return e == hipSuccess ? TEUK_OK : TEUK_EDEVICE;
}

}  // namespace lwk

extern "C" int teuk_arith_host(int words, int op, const double *a, const double *b, double *out, int n) {
    if (!a || !b || !out || n < 0 || op < 0 || op > 9) return TEUK_EINVAL;
    switch (words) {
        case 1: lwk::arith_host<double>(op, a, b, out, n); return TEUK_OK;
        case 2: lwk::arith_host<lwk::dd>(op, a, b, out, n); return TEUK_OK;
        case 4: lwk::arith_host<lwk::qd>(op, a, b, out, n); return TEUK_OK;
        default: return TEUK_EINVAL;
    }
}

extern "C" int teuk_arith_device(int words, int op, const double *a, const double *b, double *out, int n) {
    if (!a || !b || !out || n < 0 || op < 0 || op > 9) return TEUK_EINVAL;
    if (n == 0) return TEUK_OK;
    switch (words) {
        case 1: return lwk::arith_device<double>(op, a, b, out, n);
        case 2: return lwk::arith_device<lwk::dd>(op, a, b, out, n);
        case 4: return lwk::arith_device<lwk::qd>(op, a, b, out, n);
        default: return TEUK_EINVAL;
    }
}
