// Kernel instantiations for T = double.
#include "prec_impl.hpp"

namespace lwk {
hipError_t coef_pass_f64(CoefJob &job, hipStream_t stream) { return coef_pass<double>(job, stream); }
hipError_t coef_pass_into_f64(CoefJob &job, double *scratch, bool planes_fp64, hipStream_t stream) {
    return coef_pass_into<double>(job, scratch, planes_fp64, stream);
}
hipError_t step_f64(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream) {
    return step_launch<double>(nt, seg, onfly, lds, insts, items, nitems, parity, stream);
}
hipError_t wide_f64(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                    const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                    bool attr_only) {
    return wide_launch<double>(nt, run, cmode, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
}
hipError_t fp64_planes(int nr, int nth, const double *rf, const double *rh, const double *trig, double *cf,
                       double *ch, hipStream_t stream) {
    dim3 grid((nth + 63) / 64, 2 * nr - 1);
    coef_fp64_planes_kernel<<<grid, 64, 0, stream>>>(nr, nth, rf, rh, trig, cf, ch);
    return hipGetLastError();
}

// ---- slab sweep (lw_slab_kernel)
template <int NT, int R, int NTH>
hipError_t slab_one(int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream, int *per_cu) {
    const void *f = (const void *)lw_slab_kernel<NT, R, NTH>;
    if (mode == 0) {
        lw_slab_kernel<NT, R, NTH><<<nblocks, NT, lds, stream>>>(*a);
        return hipGetLastError();
    }
    if (mode == 2) {
        SlabArgs arg = *a;
        void *args[] = {&arg};
        return hipLaunchCooperativeKernel(f, dim3(nblocks), dim3(NT), args, (unsigned)lds, stream);
    }
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, NT, lds);
    return e;
}

template <int NT, int NTH>
hipError_t slab_r(int r, int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream, int *per_cu) {
    switch (r) {
        case 1: return slab_one<NT, 1, NTH>(mode, lds, a, nblocks, stream, per_cu);
        case 2: return slab_one<NT, 2, NTH>(mode, lds, a, nblocks, stream, per_cu);
        case 4: return slab_one<NT, 4, NTH>(mode, lds, a, nblocks, stream, per_cu);
        default: return hipErrorInvalidValue;
    }
}

template <int NTH>
hipError_t slab_nt(int nt, int r, int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream,
                   int *per_cu) {
    switch (nt) {
        case 256: return slab_r<256, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        case 512: return slab_r<512, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        case 1024: return slab_r<1024, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        default: return hipErrorInvalidValue;
    }
}

hipError_t slab_f64(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                    hipStream_t stream, int *per_cu) {
    switch (nth) {
        case 64: return slab_nt<64>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        case 128: return slab_nt<128>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        case 256: return slab_nt<256>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace lwk
