// Host-side interface between the C ABI (teuk.cpp) and the per-precision
// kernel instantiations (prec_f64.hip, prec_dd.hip, prec_qd.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lwk {

// Everything the coefficient pass of one instance needs, plus its outputs.
struct CoefJob {
    int s, m, nr, nth, reach;
    double a_over_M, mass, rstar_min, rstar_max, cfl;
    double *ch, *cf, *wt;            // device outputs (planar, see kernels.hpp)
    int onfly;                       // FP64: write radial rows + theta factors instead of planes
    double *rf, *rh, *trig;          // device outputs when onfly
    double hdt[kMaxWords], dt[kMaxWords];   // scalars written by the pass (words of T)
    double dt_lead;
};

// Runs the coefficient pass on `stream` (allocates and frees its own scratch).
hipError_t coef_pass_f64(CoefJob &job, hipStream_t stream);
hipError_t coef_pass_dd(CoefJob &job, hipStream_t stream);
hipError_t coef_pass_qd(CoefJob &job, hipStream_t stream);

// FP64 test hook: the coefficient planes rebuilt from radial rows and theta factors.
hipError_t fp64_planes(int nr, int nth, const double *rf, const double *rh, const double *trig, double *cf,
                       double *ch, hipStream_t stream);

// One step of every work item: block size nt in {64, 128, 256}.
// seg = segment length (r* nodes per work item, as in the descriptors);
// lds = dynamic LDS bytes (radial rows of the FP64 per-point mode, else 0).
hipError_t step_f64(int nt, int seg, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                    hipStream_t stream);
hipError_t step_dd(int nt, int seg, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream);
hipError_t step_qd(int nt, int seg, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream);

}  // namespace lwk
