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

hipError_t slab_f64(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                    hipStream_t stream, int *per_cu) {
    return slab_launch<double>(nt, nth, r, mode, lds, a, nblocks, stream, per_cu);
}
}  // namespace lwk
