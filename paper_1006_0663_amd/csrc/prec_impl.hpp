// Coefficient-pass driver and step launcher, templated on the number type.
// Included once per precision by prec_f64.hip / prec_dd.hip / prec_qd.hip.
#pragma once

#include "dispatch.hpp"

#pragma clang fp contract(off)

namespace lwk {

// Published centred-difference weights (numerator, denominator) for the first
// and second derivative: reach 1 (second order) and reach 5 (tenth order,
// Fornberg 1988, Table 1).
static void stencil_weights(int reach, ThetaParams &P) {
    static const int d1_r5_num[11] = {-1, 5, -5, 5, -5, 0, 5, -5, 5, -5, 1};
    static const double d1_r5_den[11] = {1260, 504, 84, 21, 6, 1, 6, 21, 84, 504, 1260};
    static const int d2_r5_num[11] = {1, -5, 5, -5, 5, -5269, 5, -5, 5, -5, 1};
    static const double d2_r5_den[11] = {3150, 1008, 126, 21, 3, 1800, 3, 21, 126, 1008, 3150};
    static const int d1_r1_num[3] = {-1, 0, 1};
    static const double d1_r1_den[3] = {2, 1, 2};
    static const int d2_r1_num[3] = {1, -2, 1};
    static const double d2_r1_den[3] = {1, 1, 1};
    for (int k = 0; k < 2 * reach + 1; ++k) {
        P.c1_num[k] = reach == 5 ? d1_r5_num[k] : d1_r1_num[k];
        P.c1_den[k] = reach == 5 ? d1_r5_den[k] : d1_r1_den[k];
        P.c2_num[k] = reach == 5 ? d2_r5_num[k] : d2_r1_num[k];
        P.c2_den[k] = reach == 5 ? d2_r5_den[k] : d2_r1_den[k];
    }
}

template <class T> static void put_words(double *dst, T v) {
    for (int w = 0; w < kMaxWords; ++w) dst[w] = w < words_of<T>::value ? mp_word(v, w) : 0.0;
}

// Grid scalars and horizon quantities of one instance, in T (computed on the
// host with the same routines the kernels use).
template <class T> struct CoefSetup {
    T rsmin, h, dth, dt, hdt, ih;
    T rp, dpm, A, B;
    RadialParams RP;
    ThetaParams TP;
    PointParams PP;
};

template <class T> CoefSetup<T> coef_setup(CoefJob &J) {
    CoefSetup<T> S{};
    const int nr = J.nr, nth = J.nth;
    S.rsmin = mp_from<T>(J.rstar_min);
    S.h = mp_div_d(mp_sub(mp_from<T>(J.rstar_max), S.rsmin), (double)(nr - 1));
    S.dth = mp_div_d(mp_const_pi<T>(), (double)nth);
    const T hmin = mp_lead(mp_sub(S.h, S.dth)) < 0.0 ? S.h : S.dth;
    S.dt = mp_mul_d(hmin, J.cfl);
    S.hdt = mp_pow2(S.dt, 0.5);
    S.ih = mp_recip(S.h);
    put_words(J.hdt, S.hdt);
    put_words(J.dt, S.dt);
    J.dt_lead = mp_lead(S.dt);
    // horizons: r+ = M + sqrt(M^2 - a^2), r- = a^2 / r+, r+ - r- = 2 sqrt(M^2 - a^2)
    const double M = J.mass, a = J.a_over_M * J.mass;
    S.RP = RadialParams{nr, nr - 1, M, a, 0, 0, 0, 0};
    S.rp = S.dpm = S.A = S.B = mp_from<T>(0.0);
    if (M != 0.0) {
        const T aT = mp_from<T>(a), MT = mp_from<T>(M);
        const T root = mp_sqrt(mp_msub(aT, aT, mp_mul(MT, MT)));     // sqrt(M^2 - a^2)
        S.rp = mp_add(MT, root);
        const T rm = mp_div(mp_mul(aT, aT), S.rp);
        S.dpm = mp_pow2(root, 2.0);
        S.A = mp_div(mp_mul_d(S.rp, 2.0 * M), S.dpm);
        S.B = mp_div(mp_mul_d(rm, 2.0 * M), S.dpm);
        S.RP.rp_d = mp_lead(S.rp);
        S.RP.dd_d = mp_lead(S.dpm);
        S.RP.A_d = mp_lead(S.A);
        S.RP.B_d = mp_lead(S.B);
    }
    S.TP = ThetaParams{};
    S.TP.nth = nth;
    S.TP.reach = J.reach;
    S.TP.s = J.s;
    S.TP.m = J.m;
    S.TP.parity = (J.m % 2 != 0) ? -1 : 1;
    stencil_weights(J.reach, S.TP);
    S.PP = PointParams{nr, nr - 1, nth, J.s, J.m, M, a};
    return S;
}

// The coefficient pass of one instance on `stream`, with its intermediate
// tables in `scratch` (coef_scratch_doubles of them, caller-owned device
// memory); allocates nothing and does not synchronise.  FP64 with J.onfly
// writes the radial rows and theta factors (J.rf, J.rh, J.trig); with
// planes_fp64 it writes them to scratch and expands them to the eight
// planes J.cf, J.ch with the per-point routine the step kernel uses;
// otherwise (and for dd, qd) the planes come from coef_point_kernel.
template <class T>
hipError_t coef_pass_into(CoefJob &J, double *scratch, bool planes_fp64, hipStream_t stream) {
    constexpr int W = words_of<T>::value;
    const int nth = J.nth, n = 2 * J.nr - 1;
    CoefSetup<T> S = coef_setup<T>(J);
    double *r_out = scratch, *d_out = scratch + (size_t)W * n;
    double *cos_out = d_out + (size_t)W * n, *sin2_out = cos_out + (size_t)W * nth;
    coef_radial_kernel<T><<<(n + 127) / 128, 128, 0, stream>>>(S.RP, S.rsmin, S.h, S.rp, S.dpm, S.A, S.B,
                                                               r_out, d_out);
    coef_theta_kernel<T><<<(nth + 63) / 64, 64, 0, stream>>>(S.TP, S.dth, cos_out, sin2_out, J.wt);
    bool rows = false;
    hipError_t ecopy = hipSuccess;
    if constexpr (W == 1) rows = J.onfly != 0 || planes_fp64;
    if (rows) {
        double *rf = J.rf, *rh = J.rh, *trig = J.trig;
        if (planes_fp64) {
            rf = sin2_out + (size_t)W * nth;
            rh = rf + (size_t)kRadRow * J.nr;
            trig = rh + (size_t)kRadRow * (J.nr - 1);
        }
        const double sh = mp_lead(S.hdt), sih = mp_lead(mp_mul(S.hdt, S.ih));
        const double sf = mp_lead(S.dt), sif = mp_lead(mp_mul(S.dt, S.ih));
        Fp64RowParams FP{J.nr, J.nr - 1, J.s, J.m, S.PP.mass, S.PP.a, sh, sih, sf, sif};
        coef_fp64_rows_kernel<<<(n + 127) / 128, 128, 0, stream>>>(FP, r_out, d_out, rf, rh);
        ecopy = hipMemcpyAsync(trig, cos_out, sizeof(double) * nth, hipMemcpyDeviceToDevice, stream);
        if (ecopy == hipSuccess)
            ecopy = hipMemcpyAsync(trig + nth, sin2_out, sizeof(double) * nth, hipMemcpyDeviceToDevice, stream);
        if (planes_fp64 && ecopy == hipSuccess) {
            dim3 grid((nth + 63) / 64, n);
            coef_fp64_planes_kernel<<<grid, 64, 0, stream>>>(J.nr, nth, rf, rh, trig, J.cf, J.ch);
        }
    } else {
        dim3 grid((nth + 63) / 64, n);
        coef_point_kernel<T><<<grid, 64, 0, stream>>>(S.PP, r_out, d_out, cos_out, sin2_out, S.hdt,
                                                       mp_mul(S.hdt, S.ih), S.dt, mp_mul(S.dt, S.ih), J.ch, J.cf);
        if constexpr (W == 2) if (J.rows_mp) {
            // multiword radial rows [node][factor][word] and theta factors
            // [cos, sin^2][word][row] for the per-point coefficient mode
            MpRowParams MP{J.nr, J.nr - 1, J.s, J.m, S.PP.mass, S.PP.a};
            coef_mp_rows_kernel<T><<<(n + 127) / 128, 128, 0, stream>>>(MP, S.hdt, mp_mul(S.hdt, S.ih), S.dt,
                                                                         mp_mul(S.dt, S.ih), r_out, d_out, J.rf,
                                                                         J.rh);
            ecopy = hipMemcpyAsync(J.trig, cos_out, sizeof(double) * 2 * (size_t)W * nth, hipMemcpyDeviceToDevice,
                                   stream);
        }
    }
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = ecopy;
    return err;
}

// The coefficient pass of teuk_create: scratch from hipMalloc, synchronous.
template <class T>
hipError_t coef_pass(CoefJob &J, hipStream_t stream) {
    constexpr int W = words_of<T>::value;
    double *scratch = nullptr;
    hipError_t err = hipMalloc((void **)&scratch, coef_scratch_doubles(W, J.nr, J.nth, false) * sizeof(double));
    if (err != hipSuccess) return err;
    err = coef_pass_into<T>(J, scratch, false, stream);
    hipError_t e2 = hipStreamSynchronize(stream);
    if (err == hipSuccess) err = e2;
    e2 = hipFree(scratch);
    if (err == hipSuccess) err = e2;
    return err;
}

// Segment lengths with a compile-time (fully unrolled) FP64 sweep
constexpr int kFixedSeg[] = {2, 3, 4, 6, 8};

template <class T, int NT, bool ONFLY>
hipError_t step_launch_nt(int seg, size_t lds, const InstDev *insts, const WorkItem *items, int nitems, int parity,
                          hipStream_t stream) {
    if constexpr (words_of<T>::value == 1) {
        switch (seg) {
#define LWK_SEG(S_)                                                                                        \
    case S_:                                                                                             \
        lw_step_kernel<T, NT, S_, ONFLY><<<nitems, NT, lds, stream>>>(insts, items, parity);           \
        return hipGetLastError();
            LWK_SEG(2)
            LWK_SEG(3)
            LWK_SEG(4)
            LWK_SEG(6)
            LWK_SEG(8)
#undef LWK_SEG
            default: break;
        }
    }
    lw_step_kernel<T, NT, 0, ONFLY><<<nitems, NT, lds, stream>>>(insts, items, parity);
    return hipGetLastError();
}

// onfly: every instance of the launch rebuilds its coefficients per point (FP64 only)
template <class T>
hipError_t step_launch(int nt, int seg, bool onfly, size_t lds, const InstDev *insts, const WorkItem *items,
                       int nitems, int parity, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    if constexpr (words_of<T>::value == 1) {
        if (onfly) switch (nt) {
            case 64: return step_launch_nt<T, 64, true>(seg, lds, insts, items, nitems, parity, stream);
            case 128: return step_launch_nt<T, 128, true>(seg, lds, insts, items, nitems, parity, stream);
            case 256: return step_launch_nt<T, 256, true>(seg, lds, insts, items, nitems, parity, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (nt) {
        case 64: return step_launch_nt<T, 64, false>(seg, lds, insts, items, nitems, parity, stream);
        case 128: return step_launch_nt<T, 128, false>(seg, lds, insts, items, nitems, parity, stream);
        case 256: return step_launch_nt<T, 256, false>(seg, lds, insts, items, nitems, parity, stream);
        default: return hipErrorInvalidValue;
    }
}

// ---- wide sweep (see lw_wide_kernel)
// one != nullptr: a one-instance launch whose arguments carry the geometry
// and state pointers (FP64; the multiword types read them from the descriptor).
// ns = steps per launch (1, or 2 and 4 for the fused forms that exist:
// runs of one column, tm <= 2, FP64 per-point coefficients or dd).
template <class T, int NT, int P, int CM, int TM, bool ONE1, int NS>
hipError_t wide_launch_one(size_t lds, const WideArgs *one, const InstDev *insts, const WorkItem *items, int nitems,
                           int parity, hipStream_t stream, bool attr_only) {
    if (attr_only)
        return hipFuncSetAttribute((const void *)lw_wide_kernel<T, NT, P, CM, TM, ONE1, NS>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ONE1)
        lw_wide_kernel<T, NT, P, CM, TM, ONE1, NS><<<nitems, NT, lds, stream>>>(
            one->uin, one->uout, one->nr, one->nth, one->segcols, nitems, insts, items, parity);
    else
        lw_wide_kernel<T, NT, P, CM, TM, ONE1, NS><<<nitems, NT, lds, stream>>>(nullptr, nullptr, 0, 0, 0, 0, insts,
                                                                                  items, parity);
    return hipGetLastError();
}

template <class T, int NT, int P, int CM, int TM>
hipError_t wide_launch_k(int ns, size_t lds, const WideArgs *one, const InstDev *insts, const WorkItem *items,
                         int nitems, int parity, hipStream_t stream, bool attr_only) {
    constexpr int W = words_of<T>::value;
    constexpr bool has_one = W == 1;
    // fused forms (2 or 4 steps per launch): dd with runs of one column and one
    // or two unrolled iterations; FP64 (per-point coefficients) with runs of
    // one column and up to four iterations, or runs of two and up to three
    constexpr bool fused = TM >= 1 && (W == 1 ? CM > 0 && (P == 1 ? TM <= 4 : TM <= 3) : W == 2 && P == 1 && TM <= 2);
    const bool o = has_one && one;
    if (ns == 1) {
        if (o) return wide_launch_one<T, NT, P, CM, TM, has_one, 1>(lds, one, insts, items, nitems, parity, stream, attr_only);
        return wide_launch_one<T, NT, P, CM, TM, false, 1>(lds, one, insts, items, nitems, parity, stream, attr_only);
    }
    if constexpr (fused) {
        if (ns == 2) {
            if (o) return wide_launch_one<T, NT, P, CM, TM, has_one, 2>(lds, one, insts, items, nitems, parity, stream, attr_only);
            return wide_launch_one<T, NT, P, CM, TM, false, 2>(lds, one, insts, items, nitems, parity, stream, attr_only);
        }
        if (ns == 4) {
            if (o) return wide_launch_one<T, NT, P, CM, TM, has_one, 4>(lds, one, insts, items, nitems, parity, stream, attr_only);
            return wide_launch_one<T, NT, P, CM, TM, false, 4>(lds, one, insts, items, nitems, parity, stream, attr_only);
        }
    }
    return hipErrorInvalidValue;
}

// unrolled variants (tm = 1..4) exist for FP64 blocks of 128..512 threads in
// the per-point coefficient modes; everything else takes the loop.
template <class T, int NT, int P, int CM>
hipError_t wide_launch_nt(int tm, int ns, size_t lds, const WideArgs *one, const InstDev *insts, const WorkItem *items,
                          int nitems, int parity, hipStream_t stream, bool attr_only) {
    // (multiword types: the unrolled forms lose ~25 % for qd, whose registers
    // they exhaust, and gain nothing for dd beyond two iterations; qd always
    // takes the loop, dd unrolls one or two iterations, which fused steps need)
    constexpr int W = words_of<T>::value;
    constexpr bool unrolled = NT >= 128 && NT <= 512 && ((W == 1 && CM > 0) || W == 2);
    if constexpr (unrolled) {
        switch (tm) {
            case 1: return wide_launch_k<T, NT, P, CM, 1>(ns, lds, one, insts, items, nitems, parity, stream, attr_only);
            case 2: return wide_launch_k<T, NT, P, CM, 2>(ns, lds, one, insts, items, nitems, parity, stream, attr_only);
            case 3:
                if constexpr (W == 1)
                    return wide_launch_k<T, NT, P, CM, 3>(ns, lds, one, insts, items, nitems, parity, stream, attr_only);
                break;
            case 4:
                if constexpr (W == 1)
                    return wide_launch_k<T, NT, P, CM, 4>(ns, lds, one, insts, items, nitems, parity, stream, attr_only);
                break;
            default: break;
        }
    }
    return wide_launch_k<T, NT, P, CM, 0>(ns, lds, one, insts, items, nitems, parity, stream, attr_only);
}

template <class T, int P, int CM>
hipError_t wide_launch_o(int nt, int tm, int ns, size_t lds, const WideArgs *one, const InstDev *insts,
                         const WorkItem *items, int nitems, int parity, hipStream_t stream, bool attr_only) {
    constexpr int W = words_of<T>::value;
    switch (nt) {
        case 64: return wide_launch_nt<T, 64, P, CM>(tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        case 128: return wide_launch_nt<T, 128, P, CM>(tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        case 256: return wide_launch_nt<T, 256, P, CM>(tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        case 512:
            if constexpr (W <= 2)
                return wide_launch_nt<T, 512, P, CM>(tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
            break;
        case 1024:
            if constexpr (W == 1 && P == 1)
                return wide_launch_nt<T, 1024, P, CM>(tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
            break;
        default: break;
    }
    return hipErrorInvalidValue;
}

// run = columns per lane and iteration (1, or 2 for FP64); cmode =
// coefficient mode of lw_wide_kernel (1 and 2 for FP64 only); tm = unrolled
// iteration count (1..4) when every work item needs at most that many, else 0;
// ns = steps per launch (see wide_launch_k)
template <class T>
hipError_t wide_launch(int nt, int run, int cmode, int tm, int ns, size_t lds, const WideArgs *one,
                       const InstDev *insts, const WorkItem *items, int nitems, int parity, hipStream_t stream,
                       bool attr_only) {
    if (!attr_only && nitems <= 0) return hipSuccess;
    if constexpr (words_of<T>::value == 1) {
#define LWK_WIDE(P_, CM_)                                                                                     \
    if (run == P_ && cmode == CM_)                                                                             \
        return wide_launch_o<T, P_, CM_>(nt, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        LWK_WIDE(1, 0)
        LWK_WIDE(1, 1)
        LWK_WIDE(1, 2)
        LWK_WIDE(2, 0)
        LWK_WIDE(2, 1)
        LWK_WIDE(2, 2)
#undef LWK_WIDE
        return hipErrorInvalidValue;
    } else {
        if (run != 1) return hipErrorInvalidValue;
        if (cmode == 0)
            return wide_launch_o<T, 1, 0>(nt, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        // planes requested one phase ahead: double-double only (quad-double
        // has no registers to spare for a second set of planes)
        if constexpr (words_of<T>::value == 2) {
            if (cmode == 3)
                return wide_launch_o<T, 1, 3>(nt, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
            if (cmode == 4)
                return wide_launch_o<T, 1, 4>(nt, tm, ns, lds, one, insts, items, nitems, parity, stream, attr_only);
        }
        return hipErrorInvalidValue;
    }
}

// ---- slab sweep (lw_slab_kernel): nt in {256, 512, 1024}, nth in {64, 128,
// 256}, r in {1, 2, 4} (FP64) or {1, 2} (double-double, quad-double)
template <class T, int NT, int R, int NTH>
hipError_t slab_one(int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream, int *per_cu) {
    const void *f = (const void *)lw_slab_kernel<T, NT, R, NTH>;
    if (mode == 0) {
        lw_slab_kernel<T, NT, R, NTH><<<nblocks, NT, lds, stream>>>(*a);
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

template <class T, int NT, int NTH>
hipError_t slab_r(int r, int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream, int *per_cu) {
    switch (r) {
        case 1: return slab_one<T, NT, 1, NTH>(mode, lds, a, nblocks, stream, per_cu);
        case 2: return slab_one<T, NT, 2, NTH>(mode, lds, a, nblocks, stream, per_cu);
        case 4:
            if constexpr (words_of<T>::value == 1) return slab_one<T, NT, 4, NTH>(mode, lds, a, nblocks, stream, per_cu);
            break;
        default: break;
    }
    return hipErrorInvalidValue;
}

template <class T, int NTH>
hipError_t slab_nt(int nt, int r, int mode, size_t lds, const SlabArgs *a, int nblocks, hipStream_t stream,
                   int *per_cu) {
    switch (nt) {
        case 256: return slab_r<T, 256, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        case 512: return slab_r<T, 512, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        case 1024: return slab_r<T, 1024, NTH>(r, mode, lds, a, nblocks, stream, per_cu);
        default: return hipErrorInvalidValue;
    }
}

template <class T>
hipError_t slab_launch(int nt, int nth, int r, int mode, size_t lds, const SlabArgs *a, int nblocks,
                       hipStream_t stream, int *per_cu) {
    switch (nth) {
        case 64: return slab_nt<T, 64>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        case 128: return slab_nt<T, 128>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        case 256: return slab_nt<T, 256>(nt, r, mode, lds, a, nblocks, stream, per_cu);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lwk
