// Kernel instantiations for T = double.
#include "prec_impl.hpp"

namespace lwk {
hipError_t coef_pass_f64(CoefJob &job, hipStream_t stream) { return coef_pass<double>(job, stream); }
hipError_t step_f64(int nt, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream) {
    return step_launch<double>(nt, insts, items, nitems, parity, stream);
}
}  // namespace lwk
