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
    int rows_mp;                     // dd: also write dd radial rows + theta factors (rf, rh, trig)
    double *rf, *rh, *trig;          // device outputs when onfly or rows_mp
    double hdt[kMaxWords], dt[kMaxWords];   // scalars written by the pass (words of T)
    double dt_lead;
};

// Runs the coefficient pass on `stream` (allocates and frees its own scratch).
hipError_t coef_pass_f64(CoefJob &job, hipStream_t stream);
hipError_t coef_pass_dd(CoefJob &job, hipStream_t stream);
hipError_t coef_pass_qd(CoefJob &job, hipStream_t stream);

// Doubles of scratch the coefficient pass of one instance needs: r and Delta
// at the n_r nodes and n_r - 1 half nodes, cos and sin^2 at the rows (all W
// words each), and for FP64 the radial rows and theta factors when the pass
// is to produce planes (coef_pass_into with planes_fp64).
inline size_t coef_scratch_doubles(int words, int nr, int nth, bool planes_fp64) {
    const size_t n = 2 * (size_t)nr - 1;
    size_t d = (size_t)words * (2 * n + 2 * (size_t)nth);
    if (planes_fp64) d += (size_t)kRadRow * n + 2 * (size_t)nth;
    return d;
}

// The same pass with caller-owned scratch (coef_scratch_doubles doubles of
// device memory): allocates nothing, does not synchronise.  planes_fp64
// (FP64 only): produce the eight planes job.cf, job.ch (via radial rows kept
// in scratch) instead of the rows.
hipError_t coef_pass_into_f64(CoefJob &job, double *scratch, bool planes_fp64, hipStream_t stream);
hipError_t coef_pass_into_dd(CoefJob &job, double *scratch, hipStream_t stream);
hipError_t coef_pass_into_qd(CoefJob &job, double *scratch, hipStream_t stream);

// FP64 test hook: the coefficient planes rebuilt from radial rows and theta factors.
hipError_t fp64_planes(int nr, int nth, const double *rf, const double *rh, const double *trig, double *cf,
                       double *ch, hipStream_t stream);

// One step of every work item: block size nt in {64, 128, 256}.
// seg = segment length (r* nodes per work item, as in the descriptors);
// onfly = every instance rebuilds its coefficients per point (FP64);
// lds = dynamic LDS bytes (radial rows of the FP64 per-point mode, else 0).
hipError_t step_f64(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                    hipStream_t stream);
hipError_t step_dd(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream);
hipError_t step_qd(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                   hipStream_t stream);

// One step of every work item with the wide sweep (lw_wide_kernel): block
// size nt in {64, 128, 256, 512 (FP64, dd), 1024 (FP64, run 1)}; run = columns
// per lane and iteration (1, or 2 for FP64); cmode = where the coefficients
// come from: 0 stored planes, 1 radial rows staged in LDS, 2 radial rows by
// scalar loads (n_theta a multiple of 64); tm = 2, 3 or 4 selects the variant
// with that many iterations unrolled and all loads issued up front (every
// work item must need at most tm iterations), 0 the loop; ns = time steps per
// launch (1; 2 or 4 for FP64 with per-point coefficients and dd, runs of one
// column, tm <= 2); one = arguments of a
// one-instance launch (or nullptr: the work list); one work item is one segment of the
// descriptor's segcols nodes; lds = dynamic LDS bytes (exchange arrays plus
// the FP64 radial rows).  attr_only: only enable `lds` bytes of dynamic LDS
// for that kernel (needed above 64 KiB), launch nothing.
hipError_t wide_f64(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                    const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                    bool attr_only);
// The persistent slab sweep (lw_slab_kernel, one instance; FP64 with
// per-point coefficients, or double-double / quad-double with stored planes):
// nt threads in {256, 512, 1024} = nt / nth groups, nth = n_theta in {64,
// 128, 256}, r in {1, 2, 4} (FP64) or {1, 2} (multiword) columns per lane
// (hipErrorInvalidValue otherwise).  mode 0: launch the nblocks blocks on
// `stream` with `lds` bytes of dynamic LDS (the caller has checked that the
// device holds them all at once); mode 2: the same as a cooperative launch
// (the runtime guarantees residency or fails); mode 1: enable `lds` bytes for
// the kernel and store in *per_cu how many of its blocks one compute unit
// holds.
hipError_t slab_f64(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                    hipStream_t stream, int *per_cu);
hipError_t slab_dd(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                   hipStream_t stream, int *per_cu);
hipError_t slab_qd(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                   hipStream_t stream, int *per_cu);
hipError_t wide_dd(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                    const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                    bool attr_only);
hipError_t wide_qd(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                    const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                    bool attr_only);

}  // namespace lwk
