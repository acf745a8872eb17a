// Kernel instantiations for T = qd.
#include "prec_impl.hpp"

namespace lwk {
hipError_t coef_pass_qd(CoefJob &job, hipStream_t stream) { return coef_pass<qd>(job, stream); }
hipError_t coef_pass_into_qd(CoefJob &job, double *scratch, hipStream_t stream) {
    return coef_pass_into<qd>(job, scratch, false, stream);
}
hipError_t step_qd(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream) {
    return step_launch<qd>(nt, seg, onfly, lds, insts, items, nitems, parity, stream);
}
hipError_t wide_qd(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                    const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                    bool attr_only) {
    return wide_launch<qd>(nt, run, cmode, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
}
hipError_t slab_qd(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                   hipStream_t stream, int *per_cu) {
    return slab_launch<qd>(nt, nth, r, mode, lds, a, nblocks, stream, per_cu);
}
}  // namespace lwk
