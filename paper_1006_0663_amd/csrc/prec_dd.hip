// Kernel instantiations for T = dd.
#include "prec_impl.hpp"

namespace lwk {
hipError_t coef_pass_dd(CoefJob &job, hipStream_t stream) { return coef_pass<dd>(job, stream); }
hipError_t step_dd(int nt, int seg, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream) {
    return step_launch<dd>(nt, seg, lds, insts, items, nitems, parity, stream);
}
}  // namespace lwk
