// gfx950 kernels of the Teukolsky Lax-Wendroff step, templated on the
// number type T (double, dd, qd).
//
// Device layout (everything "planar": one plane of doubles per real
// component and per word, theta index fastest so that a wavefront's lanes,
// which run along theta, touch consecutive addresses):
//
//   state   u[(c*W + w)][i][j]     c = Phi_R, Phi_I, Pi_R, Pi_I; i = r* node; j = theta row
//   coef    ch[(c*W + w)][i][j]    c = 0..7 at the half point r*_{i+1/2}, i < n_r - 1
//           cf[(c*W + w)][i][j]    c = 0..7 at r*_i
//             0: s/dr* b   1: s W   2,3: s/dr* K   4,5: s Ct   6,7: s C0
//             with s = dt/2 at half points (stage lw1) and s = dt at nodes (lw2)
//   weights wt[((k+R)*W + w)][j]   angular operator row j, tap k = -R..R:
//             c2_k/dth^2 + cot(th_j) c1_k/dth, times the ghost sign when row
//             j+k lies beyond a pole, plus V(th_j) on the centre tap
//
// The step kernel sweeps r* columns: a group of n_theta lanes owns one
// theta column (one lane per row) of one r* segment and walks along r*,
// keeping the previous column, its half-step values and their angular
// derivatives in registers.  The only cross-lane traffic is the 2R+1 tap
// angular stencil, exchanged through LDS once for u^n and once for
// u^{n+1/2} per column.  Each segment recomputes one column of overlap at its
// left edge, so segments are independent and one launch advances a step.
#pragma once

#include "mpdot.hpp"
#include "mpfunc.hpp"

#pragma clang fp contract(off)

namespace lwk {

constexpr int kMaxReach = 5;
constexpr int kMaxWords = 4;

// Per-instance descriptor, read by every block of the step kernel.
struct InstDev {
    int nr, nth, reach, segcols;
    int groups;                 // number of segment groups (blocks) of this instance
    int words;
    int onfly;                  // FP64 only: evaluate coefficients per point from rh/rf/trig
    double *u[2];
    const double *ch, *cf, *wt;
    const double *rh, *rf;      // radial rows (kRadRow doubles) at half nodes / nodes
    const double *trig;         // [2][nth]: cos(theta_j), sin^2(theta_j)
    double hdt[kMaxWords], dt[kMaxWords];
};

// ------------------------------------------------------------------ FP64 per-point coefficients
// For FP64 the step kernel can rebuild the eight scaled coefficients of a
// point from one row of radial factors (wave-uniform along the r* sweep) and
// cos, sin^2 of its theta row, instead of reading 16 stored doubles per
// update.  With Sigma^2 = varpi^2 - a^2 Delta sin^2, q = 1/Sigma^2, s = dt/2
// (half nodes) or dt (nodes), i = 1/dr* and
//   T1 = 2s'(r Delta - M(r^2-a^2)), T2 = 4Mamr, T3 = 2s'a Delta,
//   T4 = Delta(6 Delta/r^2 + 3(s'+1)Delta'/r), T5 = 6am Delta/r + 4ams'(r-M),
//   T6 = Delta(6 varpi/r + 2r) + varpi s' Delta', T7 = 2am varpi,
//   T8 = a^2 Delta (varpi Delta' - 4 r Delta)/2          (s' = spin weight)
// the coefficients are s i b, s W, s i K, s Ct, s C0 with b = varpi sqrt(q),
// W = Delta q, Ct = q (T1 + i(T2 + T3 cos)), C0 = q (T4 + i T5),
// Cs = q (T6 + i T7), b d_r*b = sin^2 q^2 T8, K = b d_r*b - b Ct - Cs.
constexpr int kRadRow = 16;
enum {
    kVp2, kA2D, kVp, kSD, kSIVp, kST1, kST2, kST3, kST4, kST5, kSIT1, kSIT2, kSIT3, kSIT6, kSIT7, kSIT8
};

// 1/sqrt(x), x > 0, to about one ulp: the hardware reciprocal square root
// seeds two Newton steps on the device; the host starts from 1/sqrt(x).  The
// step y(3/2 - x y^2/2) is written y + y(1/2 - x y^2/2), whose constants are
// inline operands of the FMA.
MPA double rsqrt_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rsq(x);
#else
    double y = 1.0 / sqrt(x);
#endif
    const double hx = 0.5 * x;
    y = fma(y, fma(-hx, y * y, 0.5), y);
    y = fma(y, fma(-hx, y * y, 0.5), y);
    return y;
}

// (Every operation takes at most one row value: where the rows sit in
// scalar registers, an instruction can read only one of them.)
template <class RowPtr>
MPA void coef_fp64_point(RowPtr rr, double cs, double s2, double *c) {
    const double X = rr[kVp2] - rr[kA2D] * s2;
    const double rq = rsqrt_nr(X);
    const double q = rq * rq;
    const double b = rr[kVp] * rq;
    c[0] = rr[kSIVp] * rq;
    c[1] = rr[kSD] * q;
    c[2] = q * fma(s2 * q, rr[kSIT8], -(b * rr[kSIT1] + rr[kSIT6]));
    c[3] = -q * fma(b, cs * rr[kSIT3] + rr[kSIT2], rr[kSIT7]);
    c[4] = q * rr[kST1];
    c[5] = q * (cs * rr[kST3] + rr[kST2]);
    c[6] = q * rr[kST4];
    c[7] = q * rr[kST5];
}

// radial row of location t (nodes first, then half nodes) from r and Delta
MPA void coef_fp64_radial_row(int s_, int m_, double M, double a, double r, double delta, double sg,
                              double sgi, double *row) {
    const double s = s_, m = m_;
    const double a2 = a * a, r2 = r * r, vp = r2 + a2, dd = 2.0 * (r - M), ir = 1.0 / r;
    const double T1 = 2.0 * s * fma(r, delta, -M * (r2 - a2));
    const double T2 = 4.0 * M * a * m * r;
    const double T3 = 2.0 * s * a * delta;
    const double T4 = delta * fma(3.0 * (s + 1.0) * dd, ir, 6.0 * delta * ir * ir);
    const double T5 = fma(6.0 * a * m * delta, ir, 4.0 * a * m * s * (r - M));
    const double T6 = fma(delta, fma(6.0 * vp, ir, 2.0 * r), vp * s * dd);
    const double T7 = 2.0 * a * m * vp;
    const double T8 = 0.5 * a2 * delta * fma(vp, dd, -4.0 * r * delta);
    row[kVp2] = vp * vp;
    row[kA2D] = a2 * delta;
    row[kVp] = vp;
    row[kSD] = sg * delta;
    row[kSIVp] = sgi * vp;
    row[kST1] = sg * T1;
    row[kST2] = sg * T2;
    row[kST3] = sg * T3;
    row[kST4] = sg * T4;
    row[kST5] = sg * T5;
    row[kSIT1] = sgi * T1;
    row[kSIT2] = sgi * T2;
    row[kSIT3] = sgi * T3;
    row[kSIT6] = sgi * T6;
    row[kSIT7] = sgi * T7;
    row[kSIT8] = sgi * T8;
}

struct Fp64RowParams {
    int n_full, n_half, s, m;
    double mass, a, s_half, si_half, s_full, si_full;
};

static __global__ void coef_fp64_rows_kernel(Fp64RowParams P, const double *r_in, const double *delta_in,
                                      double *rf, double *rh) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n_full + P.n_half;
    if (t >= n) return;
    const bool half = t >= P.n_full;
    double *row = half ? rh + (size_t)(t - P.n_full) * kRadRow : rf + (size_t)t * kRadRow;
    coef_fp64_radial_row(P.s, P.m, P.mass, P.a, r_in[t], delta_in[t], half ? P.s_half : P.s_full,
                         half ? P.si_half : P.si_full, row);
}

// the planes of the test hook, from the same per-point routine the kernel uses
static __global__ void coef_fp64_planes_kernel(int nr, int nth, const double *rf, const double *rh, const double *trig,
                                        double *cf, double *ch) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (j >= nth || t >= 2 * nr - 1) return;
    const bool half = t >= nr;
    const int i = half ? t - nr : t;
    const int ni = half ? nr - 1 : nr;
    double c[8];
    coef_fp64_point((half ? rh : rf) + (size_t)i * kRadRow, trig[j], trig[nth + j], c);
    double *out = half ? ch : cf;
    const size_t plane = (size_t)ni * nth;
    for (int k = 0; k < 8; ++k) out[(size_t)k * plane + (size_t)i * nth + j] = c[k];
}

struct WorkItem {
    int inst;
    int group;
};

template <class T> MPA T ld(const double *p, size_t plane, size_t idx) {
    T v;
    for (int w = 0; w < words_of<T>::value; ++w) mp_set_word(v, w, p[w * plane + idx]);
    return v;
}
template <class T> MPA void st(double *p, size_t plane, size_t idx, T v) {
    for (int w = 0; w < words_of<T>::value; ++w) p[w * plane + idx] = mp_word(v, w);
}
template <class T> MPA T from_words(const double *w) {
    T v;
    for (int k = 0; k < words_of<T>::value; ++k) mp_set_word(v, k, w[k]);
    return v;
}

// Device loads and stores through global-address-space pointers with 32-bit
// offsets.  Pointers read from the descriptors are generic; without the
// address space the compiler emits FLAT instructions, which count against
// the LDS wait counter too, so every LDS wait would also wait for every
// outstanding HBM load.
#define GLB __attribute__((address_space(1)))
#define CNS __attribute__((address_space(4)))     // constant: uniform addresses become scalar loads
__device__ __forceinline__ const GLB double *gptr(const double *p) { return (const GLB double *)p; }
__device__ __forceinline__ GLB double *gptr(double *p) { return (GLB double *)p; }
template <class T> __device__ __forceinline__ T gld(const GLB double *p, uint32_t plane, uint32_t idx) {
    T v;
#pragma unroll
    for (int w = 0; w < words_of<T>::value; ++w) mp_set_word(v, w, p[w * plane + idx]);
    return v;
}
template <class T> __device__ __forceinline__ void gst(GLB double *p, uint32_t plane, uint32_t idx, const T &v) {
#pragma unroll
    for (int w = 0; w < words_of<T>::value; ++w) p[w * plane + idx] = mp_word(v, w);
}

// ------------------------------------------------------------------ multiword per-point coefficients
// The radial row of kernels' per-point mode in working precision T: the same
// sixteen factors as coef_fp64_radial_row (kVp2 .. kSIT8), each T, stored
// [node][factor][word] (16 W doubles per node), computed from r and Delta
// in T.  Products with a are taken in T; the other factors (2s, 4Mm, 6m, ...)
// are small integers, exact in double.
template <class T>
MPA void coef_radial_row_mp(int s_, int m_, double M, double a_d, const T &r, const T &delta, const T &sg,
                            const T &sgi, T *row) {
    const double s = s_, m = m_;
    const T a = mp_from<T>(a_d);
    const T a2 = mp_mul(a, a), r2 = mp_mul(r, r), vp = mp_add(r2, a2);
    const T rm = mp_sub(r, mp_from<T>(M));                    // r - M;  Delta' = 2 (r - M)
    const T ddl = mp_pow2(rm, 2.0);
    const T ir = mp_recip(r);
    const T T1 = mp_mul_d(mp_msub(mp_from<T>(M), mp_sub(r2, a2), mp_mul(r, delta)), 2.0 * s);
    const T T2 = mp_mul(mp_mul_d(r, 4.0 * M * m), a);
    const T T3 = mp_mul(mp_mul_d(delta, 2.0 * s), a);
    const T T4 = mp_mul(mp_mul(delta, ir), mp_add(mp_mul_d(ddl, 3.0 * (s + 1.0)), mp_mul_d(mp_mul(delta, ir), 6.0)));
    const T T5 = mp_mul(mp_add(mp_mul_d(mp_mul(delta, ir), 6.0 * m), mp_mul_d(rm, 4.0 * m * s)), a);
    const T T6 = mp_madd(delta, mp_madd(mp_mul_d(vp, 6.0), ir, mp_pow2(r, 2.0)), mp_mul_d(mp_mul(vp, ddl), s));
    const T T7 = mp_mul(mp_mul_d(vp, 2.0 * m), a);
    const T T8 = mp_pow2(mp_mul(mp_mul(a2, delta), mp_msub(mp_pow2(r, 4.0), delta, mp_mul(vp, ddl))), 0.5);
    row[kVp2] = mp_mul(vp, vp);
    row[kA2D] = mp_mul(a2, delta);
    row[kVp] = vp;
    row[kSD] = mp_mul(sg, delta);
    row[kSIVp] = mp_mul(sgi, vp);
    row[kST1] = mp_mul(sg, T1);
    row[kST2] = mp_mul(sg, T2);
    row[kST3] = mp_mul(sg, T3);
    row[kST4] = mp_mul(sg, T4);
    row[kST5] = mp_mul(sg, T5);
    row[kSIT1] = mp_mul(sgi, T1);
    row[kSIT2] = mp_mul(sgi, T2);
    row[kSIT3] = mp_mul(sgi, T3);
    row[kSIT6] = mp_mul(sgi, T6);
    row[kSIT7] = mp_mul(sgi, T7);
    row[kSIT8] = mp_mul(sgi, T8);
}

struct MpRowParams {
    int n_full, n_half, s, m;
    double mass, a;
};

// rows of every node (t < n_full) and half node; r and Delta planar [word][t]
template <class T>
__global__ void coef_mp_rows_kernel(MpRowParams P, T s_half, T si_half, T s_full, T si_full, const double *r_in,
                                    const double *delta_in, double *rf, double *rh) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = P.n_full + P.n_half;
    if (t >= n) return;
    constexpr int W = words_of<T>::value;
    const bool half = t >= P.n_full;
    T row[kRadRow];
    coef_radial_row_mp<T>(P.s, P.m, P.mass, P.a, ld<T>(r_in, (size_t)n, (size_t)t), ld<T>(delta_in, (size_t)n, (size_t)t),
                          half ? s_half : s_full, half ? si_half : si_full, row);
    double *out = half ? rh + (size_t)(t - P.n_full) * kRadRow * W : rf + (size_t)t * kRadRow * W;
    for (int k = 0; k < kRadRow; ++k)
        for (int w = 0; w < W; ++w) out[k * W + w] = mp_word(row[k], w);
}

// 1/sqrt(x) in double-double: the FP64 value (about one ulp) refined by one
// Newton step y + y (1 - x y^2) / 2 evaluated in double-double, which
// squares its relative error.
MPA dd rsqrt_dd(const dd &x) {
    const double y0 = rsqrt_nr(x.x0);
    dd y2;
    two_prod(y0, y0, y2.x0, y2.x1);                            // y0^2 exactly
    const dd e = mp_msub(x, y2, mp_from<dd>(1.0));             // 1 - x y0^2
    return mp_add(mp_from<dd>(y0), mp_mul_d(e, 0.5 * y0));
}

// The eight scaled coefficients of a point from its double-double radial row
// (16 dd factors at row, [factor][word]) and cos, sin^2 of its theta row:
// the terms of coef_fp64_point in double-double.
template <class RowPtr>
MPA void coef_dd_point(RowPtr row, const dd &cs, const dd &s2, dd *c) {
    auto f = [&](int k) { return dd{row[2 * k], row[2 * k + 1]}; };
    const dd X = mp_msub(f(kA2D), s2, f(kVp2));
    const dd rq = rsqrt_dd(X);
    const dd q = mp_mul(rq, rq);
    const dd b = mp_mul(f(kVp), rq);
    c[0] = mp_mul(f(kSIVp), rq);
    c[1] = mp_mul(f(kSD), q);
    c[2] = mp_mul(q, mp_sub(mp_mul(mp_mul(s2, q), f(kSIT8)), mp_madd(b, f(kSIT1), f(kSIT6))));
    c[3] = mp_neg(mp_mul(q, mp_madd(b, mp_madd(cs, f(kSIT3), f(kSIT2)), f(kSIT7))));
    c[4] = mp_mul(q, f(kST1));
    c[5] = mp_mul(q, mp_madd(cs, f(kST3), f(kST2)));
    c[6] = mp_mul(q, f(kST4));
    c[7] = mp_mul(q, f(kST5));
}

// ------------------------------------------------------------------ coefficient pass
struct RadialParams {
    int n_full, n_half;
    double mass, a;
    double rp_d, dd_d, A_d, B_d;   // leading words: r_plus, r_plus - r_minus, 2M r+/(r+-r-), 2M r-/(r+-r-)
};

// r(r*) at every node and half node: solves r*(r_plus + x) = r* for
// x = r - r_plus > 0, keeping x (not r) as the unknown so that
// Delta = x (x + r_plus - r_minus) keeps full relative precision at the
// horizon end of the grid.  Outputs r and Delta (T, planar, n_full + n_half).
template <class T>
MPA void coef_radial_one(const RadialParams &P, int t, T rsmin, T h, T rp, T dpm, T A, T B,
                         double *r_out, double *delta_out) {
    const int n = P.n_full + P.n_half;
    const double idx = t < P.n_full ? (double)t : (double)(t - P.n_full) + 0.5;
    const T rs = mp_madd(mp_from<T>(idx), h, rsmin);          // idx has <= 15 significant bits: exact in T
    T r, delta;
    if (P.mass == 0.0) {                                       // flat space: r* = r, a = 0
        r = rs;
        delta = mp_mul(r, r);
    } else {
        const double M = P.mass, rsd = mp_lead(rs), l2m = log(2.0 * M);
        // double precision: bisection then Newton on y = ln x
        auto f = [&](double y) {
            const double x = exp(y);
            return P.rp_d + x + P.A_d * (y - l2m) - P.B_d * log((x + P.dd_d) / (2.0 * M)) - rsd;
        };
        double lo = -740.0, hi = 40.0;
        for (int it = 0; it < 80; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (f(mid) > 0.0) hi = mid; else lo = mid;
        }
        double x_d = exp(0.5 * (lo + hi));
        T x = mp_from<T>(x_d);
        const double inv2m = 1.0 / (2.0 * M);
        for (int it = 0; it < words_of<T>::value + 1; ++it) {
            // f(x) = r+ + x + A ln(x/2M) - B ln((x + d)/2M) - r*  in T;  f'(x) = 1 + A/x - B/(x+d) in double
            T fx = mp_add(rp, x);
            fx = mp_madd(A, mp_log(mp_mul_d(x, inv2m)), fx);
            if (P.B_d != 0.0) fx = mp_msub(B, mp_log(mp_mul_d(mp_add(x, dpm), inv2m)), fx);
            fx = mp_sub(fx, rs);
            const double xd = mp_lead(x);
            const double fp = 1.0 + P.A_d / xd - P.B_d / (xd + P.dd_d);
            x = mp_sub(x, mp_mul_d(fx, 1.0 / fp));
        }
        r = mp_add(rp, x);
        delta = mp_mul(x, mp_add(x, dpm));
    }
    st(r_out, (size_t)n, (size_t)t, r);
    st(delta_out, (size_t)n, (size_t)t, delta);
}

template <class T>
__global__ void coef_radial_kernel(RadialParams P, T rsmin, T h, T rp, T dpm, T A, T B,
                                   double *r_out, double *delta_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < P.n_full + P.n_half) coef_radial_one<T>(P, t, rsmin, h, rp, dpm, A, B, r_out, delta_out);
}

struct ThetaParams {
    int nth, reach, s, m, parity;
    int c1_num[2 * kMaxReach + 1], c2_num[2 * kMaxReach + 1];
    double c1_den[2 * kMaxReach + 1], c2_den[2 * kMaxReach + 1];
};

// Per theta row: cos, sin^2 (for the point kernel) and the folded angular weights.
template <class T>
MPA void coef_theta_one(const ThetaParams &P, int j, T dth, double *cos_out, double *sin2_out, double *wt) {
    const T th = mp_mul(mp_from<T>((double)j + 0.5), dth);   // (j + 1/2) dth
    const T x = mp_sub(th, mp_pow2(mp_const_pi<T>(), 0.5));  // theta - pi/2 in (-pi/2, pi/2)
    T sx, cx_;
    mp_sincos(x, sx, cx_);
    const T cost = mp_neg(sx), sint = cx_;
    const T sin2 = mp_mul(sint, sint);
    const T cot = mp_div(cost, sint);
    // V = s - (m + s cos)^2 / sin^2
    const T mc = mp_madd(mp_from<T>((double)P.s), cost, mp_from<T>((double)P.m));
    const T V = mp_sub(mp_from<T>((double)P.s), mp_div(mp_mul(mc, mc), sin2));
    const T idth = mp_recip(dth);
    const T idth2 = mp_mul(idth, idth);
    const int R = P.reach, W = words_of<T>::value;
    for (int k = -R; k <= R; ++k) {
        const T c2 = mp_div_d(mp_from<T>((double)P.c2_num[k + R]), P.c2_den[k + R]);
        const T c1 = mp_div_d(mp_from<T>((double)P.c1_num[k + R]), P.c1_den[k + R]);
        T w = mp_madd(mp_mul(cot, c1), idth, mp_mul(c2, idth2));
        const int q = j + k;
        if ((q < 0 || q >= P.nth) && P.parity < 0) w = mp_neg(w);
        if (k == 0) w = mp_add(w, V);
        for (int ww = 0; ww < W; ++ww) wt[((size_t)(k + R) * W + ww) * P.nth + j] = mp_word(w, ww);
    }
    st(cos_out, (size_t)P.nth, (size_t)j, cost);
    st(sin2_out, (size_t)P.nth, (size_t)j, sin2);
}

template <class T>
__global__ void coef_theta_kernel(ThetaParams P, T dth, double *cos_out, double *sin2_out, double *wt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P.nth) coef_theta_one<T>(P, j, dth, cos_out, sin2_out, wt);
}

struct PointParams {
    int n_full, n_half, nth, s, m;
    double mass, a;
};

// The eight scaled coefficients at every (node, row).  With
// varpi = r^2 + a^2, Sigma^2 = varpi^2 - a^2 Delta sin^2, q = 1/Sigma^2:
//   b = varpi sqrt(q), W = Delta q,
//   Ct = q [2s(r Delta - M(r^2 - a^2)) + i(4 M a m r + 2 s a Delta cos)],
//   C0 = W [6 Delta/r^2 + 3 (s+1) Delta'/r] + i [6 a m W / r + 4 a m s (r - M) q],
//   Cs = W (6 varpi/r + 2r) + q varpi (s Delta' + 2 i a m),
//   b d_r* b = a^2 Delta sin^2 (varpi Delta' - 4 r Delta) q^2 / 2,
//   K = b d_r* b - b Ct - Cs,   Delta' = 2 (r - M).
template <class T>
MPA void coef_point_one(const PointParams &P, int t, int j, const double *r_in, const double *delta_in,
                        const double *cos_in, const double *sin2_in, T s_half, T si_half,
                        T s_full, T si_full, double *ch, double *cf) {
    const int n = P.n_full + P.n_half;
    const T r = ld<T>(r_in, (size_t)n, (size_t)t);
    const T delta = ld<T>(delta_in, (size_t)n, (size_t)t);
    const T cost = ld<T>(cos_in, (size_t)P.nth, (size_t)j);
    const T sin2 = ld<T>(sin2_in, (size_t)P.nth, (size_t)j);
    const double M = P.mass, a = P.a, s = (double)P.s, m = (double)P.m;
    // Products with a are taken in T; the other factors (2s, 4Mm, 6m, ...) are
    // small integers, exact in double.
    const T aT = mp_from<T>(a);
    const T a2 = mp_mul(aT, aT);
    const T r2 = mp_mul(r, r);
    const T varpi = mp_add(r2, a2);
    const T ddelta = mp_pow2(mp_sub(r, mp_from<T>(M)), 2.0);
    const T ad2 = mp_mul(mp_mul(a2, delta), sin2);            // a^2 Delta sin^2
    const T sig2 = mp_msub(mp_from<T>(1.0), ad2, mp_mul(varpi, varpi));
    const T q = mp_recip(sig2);
    const T b = mp_mul(varpi, mp_sqrt(q));
    const T W = mp_mul(delta, q);
    const T ir = mp_recip(r);
    // Ct
    const T ct_re = mp_mul(q, mp_mul_d(mp_msub(mp_from<T>(M), mp_sub(r2, a2), mp_mul(r, delta)), 2.0 * s));
    const T ct_im = mp_mul(q, mp_mul_d(mp_madd(mp_mul_d(delta, 2.0 * s), cost, mp_mul_d(r, 4.0 * M * m)), a));
    // C0
    const T c0_re = mp_mul(W, mp_madd(mp_mul_d(ddelta, 3.0 * (s + 1.0)), ir, mp_mul_d(mp_mul(delta, mp_mul(ir, ir)), 6.0)));
    const T c0_im = mp_mul_d(mp_add(mp_mul_d(mp_mul(W, ir), 6.0 * m),
                                    mp_mul(q, mp_mul_d(mp_sub(r, mp_from<T>(M)), 4.0 * m * s))), a);
    // Cs
    const T cs_re = mp_madd(W, mp_madd(mp_mul_d(varpi, 6.0), ir, mp_pow2(r, 2.0)),
                            mp_mul(mp_mul(q, varpi), mp_mul_d(ddelta, s)));
    const T cs_im = mp_mul_d(mp_mul_d(mp_mul(q, varpi), 2.0 * m), a);
    // b d_r* b
    const T bdb = mp_pow2(mp_mul(mp_mul(ad2, mp_msub(mp_pow2(r, 4.0), delta, mp_mul(varpi, ddelta))), mp_mul(q, q)), 0.5);
    // K = bdb - b Ct - Cs
    const T k_re = mp_sub(mp_msub(b, ct_re, bdb), cs_re);
    const T k_im = mp_neg(mp_add(mp_mul(b, ct_im), cs_im));
    const bool half = t >= P.n_full;
    const int i = half ? t - P.n_full : t;
    const int nr_loc = half ? P.n_half : P.n_full;
    const T sg = half ? s_half : s_full, sgi = half ? si_half : si_full;
    double *out = half ? ch : cf;
    const size_t plane = (size_t)nr_loc * P.nth, idx = (size_t)i * P.nth + j;
    const int Wd = words_of<T>::value;
    const T vals[8] = {mp_mul(sgi, b), mp_mul(sg, W), mp_mul(sgi, k_re), mp_mul(sgi, k_im),
                       mp_mul(sg, ct_re), mp_mul(sg, ct_im), mp_mul(sg, c0_re), mp_mul(sg, c0_im)};
    for (int c = 0; c < 8; ++c) st(out + (size_t)c * Wd * plane, plane, idx, vals[c]);
}

template <class T>
__global__ void coef_point_kernel(PointParams P, const double *r_in, const double *delta_in,
                                  const double *cos_in, const double *sin2_in, T s_half, T si_half,
                                  T s_full, T si_full, double *ch, double *cf) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (j < P.nth && t < P.n_full + P.n_half)
        coef_point_one<T>(P, t, j, r_in, delta_in, cos_in, sin2_in, s_half, si_half, s_full, si_full, ch, cf);
}

// ------------------------------------------------------------------ step kernel
template <class T> struct Pt {
    cx<T> phi, pi;
};

// one stage of the scheme at one point:
//   out_Phi = base_Phi - B dPhi + s Pibar
//   out_Pi  = base_Pi  + B dPi - K dPhi + W Lbar + C0 Phibar - Ct Pibar
// with bar = neighbour average, d = neighbour difference, coefficients
// pre-scaled by s (= dt/2 or dt) and 1/dr*; for (lw1) base = bar.  Each of
// the four real outputs is one fused dot product (see mpdot.hpp).
template <class T>
MPA Pt<T> lw_stage(const Pt<T> &base, const Pt<T> &bar, const Pt<T> &d, const cx<T> &lbar, const T *c,
                   const T &s) {
    const T nB = mp_neg(c[0]), nKr = mp_neg(c[2]), nKi = mp_neg(c[3]);
    const T nCr = mp_neg(c[4]), nCi = mp_neg(c[5]), nDi = mp_neg(c[7]);
    Pt<T> o;
    {
        Acc<T> a;
        a.value(base.phi.re);
        a.prod(nB, d.phi.re);
        a.prod(s, bar.pi.re);
        o.phi.re = a.result();
    }
    {
        Acc<T> a;
        a.value(base.phi.im);
        a.prod(nB, d.phi.im);
        a.prod(s, bar.pi.im);
        o.phi.im = a.result();
    }
    {
        Acc<T> a;                                   // Re: + B dPi - K dPhi + W L + C0 Phi - Ct Pi
        a.value(base.pi.re);
        a.prod(c[0], d.pi.re);
        a.prod(nKr, d.phi.re);
        a.prod(c[3], d.phi.im);
        a.prod(c[1], lbar.re);
        a.prod(c[6], bar.phi.re);
        a.prod(nDi, bar.phi.im);
        a.prod(nCr, bar.pi.re);
        a.prod(c[5], bar.pi.im);
        o.pi.re = a.result();
    }
    {
        Acc<T> a;                                   // Im
        a.value(base.pi.im);
        a.prod(c[0], d.pi.im);
        a.prod(nKr, d.phi.im);
        a.prod(nKi, d.phi.re);
        a.prod(c[1], lbar.im);
        a.prod(c[6], bar.phi.im);
        a.prod(c[7], bar.phi.re);
        a.prod(nCr, bar.pi.im);
        a.prod(nCi, bar.pi.re);
        o.pi.im = a.result();
    }
    return o;
}

// FP64 stage with the coefficients built from the radial row rr at the point
// (the per-point coefficient modes): the terms of coef_fp64_point followed by
// lw_stage, except that q = 1/X, a factor of every Pi-row coefficient but B,
// multiplies their sum once instead of each coefficient (seven products fewer
// per stage, two more).  Writing K = q (kr + i ki), C_t = q (ST1 + i ci),
// W = q SD, C0 = q (ST4 + i ST5):
//   out_Pi = base_Pi + B dPi + q (-(kr + i ki) dPhi + SD Lbar + (ST4 + i ST5) Phibar
//                                 - (ST1 + i ci) Pibar)
template <class RowPtr>
MPA Pt<double> lw_stage_row(const Pt<double> &base, const Pt<double> &bar, const Pt<double> &d,
                            const cx<double> &lbar, RowPtr rr, double cs, double s2, double s) {
    const double X = rr[kVp2] - rr[kA2D] * s2;
    const double rq = rsqrt_nr(X);
    const double q = rq * rq;
    const double b = rr[kVp] * rq;
    const double B = rr[kSIVp] * rq;
    const double kr = fma(s2 * q, rr[kSIT8], -(b * rr[kSIT1] + rr[kSIT6]));
    const double ki = -fma(b, cs * rr[kSIT3] + rr[kSIT2], rr[kSIT7]);
    const double ci = cs * rr[kST3] + rr[kST2];
    Pt<double> o;
    o.phi.re = fma(s, bar.pi.re, fma(-B, d.phi.re, base.phi.re));
    o.phi.im = fma(s, bar.pi.im, fma(-B, d.phi.im, base.phi.im));
    double sr = -kr * d.phi.re;
    sr = fma(ki, d.phi.im, sr);
    sr = fma(rr[kSD], lbar.re, sr);
    sr = fma(rr[kST4], bar.phi.re, sr);
    sr = fma(-rr[kST5], bar.phi.im, sr);
    sr = fma(-rr[kST1], bar.pi.re, sr);
    sr = fma(ci, bar.pi.im, sr);
    double si = -kr * d.phi.im;
    si = fma(-ki, d.phi.re, si);
    si = fma(rr[kSD], lbar.im, si);
    si = fma(rr[kST4], bar.phi.im, si);
    si = fma(rr[kST5], bar.phi.re, si);
    si = fma(-rr[kST1], bar.pi.im, si);
    si = fma(-ci, bar.pi.re, si);
    o.pi.re = fma(q, sr, fma(B, d.pi.re, base.pi.re));
    o.pi.im = fma(q, si, fma(B, d.pi.im, base.pi.im));
    return o;
}

template <class T>
MPA Pt<T> ld_pt(const double *u, size_t plane, size_t idx) {
    constexpr int W = words_of<T>::value;
    Pt<T> p;
    p.phi.re = ld<T>(u + 0 * W * plane, plane, idx);
    p.phi.im = ld<T>(u + 1 * W * plane, plane, idx);
    p.pi.re = ld<T>(u + 2 * W * plane, plane, idx);
    p.pi.im = ld<T>(u + 3 * W * plane, plane, idx);
    return p;
}
template <class T>
MPA void st_pt(double *u, size_t plane, size_t idx, const Pt<T> &p) {
    constexpr int W = words_of<T>::value;
    st(u + 0 * W * plane, plane, idx, p.phi.re);
    st(u + 1 * W * plane, plane, idx, p.phi.im);
    st(u + 2 * W * plane, plane, idx, p.pi.re);
    st(u + 3 * W * plane, plane, idx, p.pi.im);
}

template <class T> __device__ __forceinline__ Pt<T> gld_pt(const GLB double *u, uint32_t plane, uint32_t idx) {
    constexpr uint32_t W = words_of<T>::value;
    Pt<T> p;
    p.phi.re = gld<T>(u, plane, idx);
    p.phi.im = gld<T>(u + 1 * W * plane, plane, idx);
    p.pi.re = gld<T>(u + 2 * W * plane, plane, idx);
    p.pi.im = gld<T>(u + 3 * W * plane, plane, idx);
    return p;
}
template <class T> __device__ __forceinline__ void gst_pt(GLB double *u, uint32_t plane, uint32_t idx, const Pt<T> &p) {
    constexpr uint32_t W = words_of<T>::value;
    gst(u, plane, idx, p.phi.re);
    gst(u + 1 * W * plane, plane, idx, p.phi.im);
    gst(u + 2 * W * plane, plane, idx, p.pi.re);
    gst(u + 3 * W * plane, plane, idx, p.pi.im);
}

template <class T> MPA cx<T> c_avg(const cx<T> &a, const cx<T> &b) {
    return {mp_pow2(mp_add_fast(a.re, b.re), 0.5), mp_pow2(mp_add_fast(a.im, b.im), 0.5)};
}
template <class T> MPA cx<T> c_diff(const cx<T> &a, const cx<T> &b) {     // b - a
    return {mp_add_fast(b.re, mp_neg(a.re)), mp_add_fast(b.im, mp_neg(a.im))};
}
template <class T> MPA Pt<T> pt_avg(const Pt<T> &a, const Pt<T> &b) { return {c_avg(a.phi, b.phi), c_avg(a.pi, b.pi)}; }
template <class T> MPA Pt<T> pt_diff(const Pt<T> &a, const Pt<T> &b) { return {c_diff(a.phi, b.phi), c_diff(a.pi, b.pi)}; }

// ---- LDS exchange of theta columns
// A complex value of T is 2W doubles, stored as W 16-byte chunks, each chunk
// in its own [lane] array: consecutive lanes touch consecutive 16-byte words,
// so a 16-byte read per lane is free of bank conflicts for every W.
struct __align__(16) d2 {
    double a, b;
};

template <class T> __device__ __forceinline__ void xput(d2 *base, int stride, int slot, const cx<T> &v) {
    constexpr int W = words_of<T>::value;
    if constexpr (W == 1) {
        base[slot] = {v.re, v.im};
    } else {
#pragma unroll
        for (int c = 0; c < W / 2; ++c) {
            base[(size_t)c * stride + slot] = {mp_word(v.re, 2 * c), mp_word(v.re, 2 * c + 1)};
            base[(size_t)(c + W / 2) * stride + slot] = {mp_word(v.im, 2 * c), mp_word(v.im, 2 * c + 1)};
        }
    }
}
template <class T> __device__ __forceinline__ cx<T> xget(const d2 *base, int stride, int slot) {
    constexpr int W = words_of<T>::value;
    cx<T> v;
    if constexpr (W == 1) {
        const d2 x = base[slot];
        v.re = x.a;
        v.im = x.b;
    } else {
#pragma unroll
        for (int c = 0; c < W / 2; ++c) {
            const d2 x = base[(size_t)c * stride + slot], y = base[(size_t)(c + W / 2) * stride + slot];
            mp_set_word(v.re, 2 * c, x.a);
            mp_set_word(v.re, 2 * c + 1, x.b);
            mp_set_word(v.im, 2 * c, y.a);
            mp_set_word(v.im, 2 * c + 1, y.b);
        }
    }
    return v;
}

// Reflected source row of tap k for row j (ghost rows mirror across the pole).
__device__ __forceinline__ int tap_row(int j, int k, int nth) {
    const int q = j + k;
    return q < 0 ? -1 - q : (q >= nth ? 2 * nth - 1 - q : q);
}

// Angular operator at row j of the column held in an exchange buffer (group
// base `base`, chunk stride `stride`): folded weights of row j times the
// reflected rows, as one fused dot product per component.  For double the
// weights (w) and source rows (qrow) of the lane are held in registers; the
// multiword types read the weights from the table and use a rolled loop.
template <class T>
__device__ __forceinline__ cx<T> theta_stencil(const d2 *base, int stride, int j, int nth, int reach,
                                               const GLB double *__restrict__ wt, const double *w, const int *qrow) {
    constexpr int W = words_of<T>::value;
    Acc<T> re, im;
    if constexpr (W == 1) {
#pragma unroll
        for (int k = 0; k < 2 * kMaxReach + 1; ++k) {
            // taps beyond the reach carry weight 0 and row 0: adding their
            // exact zero products costs less than branching around them
            const cx<T> x = xget<T>(base, stride, qrow[k]);
            re.prod(w[k], x.re);
            im.prod(w[k], x.im);
        }
    } else {
#pragma unroll 1
        for (int k = -reach; k <= reach; ++k) {
            const cx<T> x = xget<T>(base, stride, tap_row(j, k, nth));
            const T wk = gld<T>(wt + (uint32_t)((k + reach) * W * nth), (uint32_t)nth, (uint32_t)j);
            re.prod(wk, x.re);
            im.prod(wk, x.im);
        }
    }
    return {re.result(), im.result()};
}

// eight coefficients of node/half node idx at its row, from the stored planes
template <class T>
__device__ __forceinline__ void load_coef(const GLB double *planes, uint32_t plane, uint32_t idx, T *c) {
    constexpr uint32_t W = words_of<T>::value;
#pragma unroll
    for (int q = 0; q < 8; ++q) c[q] = gld<T>(planes + q * W * plane, plane, idx);
}

// one stage at node/half node idx: coefficients from the stored planes, or
// (FP64 per-point mode, ONFLY) the radial row staged in LDS
template <class T, bool ONFLY>
__device__ __forceinline__ Pt<T> stage_at(const GLB double *planes, const double *lrow, uint32_t plane,
                                          uint32_t idx, double cs, double s2, const Pt<T> &base, const Pt<T> &bar,
                                          const Pt<T> &d, const cx<T> &lbar, const T &s) {
    if constexpr (words_of<T>::value == 1 && ONFLY) {
        return lw_stage_row(base, bar, d, lbar, lrow, cs, s2, s);
    } else {
        T c[8];
        load_coef<T>(planes, plane, idx, c);
        return lw_stage(base, bar, d, lbar, c, s);
    }
}

// LDS bytes the FP64 per-point mode needs for a block of NT threads
MPA size_t rows_lds_bytes(int nt, int nth, int segcols) {
    const int G = nt / nth;
    return (size_t)(2 * G * segcols + 3) * kRadRow * sizeof(double);
}

// One full step (lw1 + lw2) of every work item.  A group of n_theta lanes
// sweeps the r* nodes a..e of its segment.  Iteration k handles column
// c = a + k: one LDS exchange carries both u^n at column c and the half-step
// value at c - 3/2 (computed in iteration k-1), so each column costs one
// barrier; then stage 2 at node c - 2 and stage 1 at half node c - 1/2.
// Double-buffered exchange slots make one barrier per iteration sufficient.
#ifndef LWK_STEP_OCC
#define LWK_STEP_OCC
#endif
template <class T, int NT, int SEG, bool ONFLY>
__global__ __launch_bounds__(NT) LWK_STEP_OCC void lw_step_kernel(const InstDev *__restrict__ insts,
                                                     const WorkItem *__restrict__ items, int parity) {
    // SEG > 0: the segment length is a compile-time constant (must equal the
    // descriptor's segcols); the sweep is then fully unrolled and every
    // column of the segment is requested from memory up front.
    constexpr int W = words_of<T>::value;
    constexpr int CH = W == 1 ? 1 : W;                 // 16-byte chunks per complex value
    __shared__ d2 xb[2][2][CH][NT];                    // [set][P = u^n, H = half step][chunk][lane]
    extern __shared__ double lrows[];                  // FP64 per-point mode: radial rows of the block
    const WorkItem wi = items[blockIdx.x];
    const InstDev &I = insts[wi.inst];
    const int nr = I.nr, nth = I.nth, R = I.reach, S = SEG > 0 ? SEG : I.segcols;
    const int G = NT / nth;
    const int g = threadIdx.x / nth, j = threadIdx.x - g * nth;
    const bool lane_on = g < G;
    const int seg = wi.group * G + g;
    const int c0 = seg * S, c1 = min(c0 + S, nr);
    const bool seg_on = lane_on && c0 < nr;
    const GLB double *uin = gptr((const double *)I.u[parity]);
    GLB double *uout = gptr(I.u[parity ^ 1]);
    const GLB double *wtab = gptr(I.wt);
    const uint32_t plane = (uint32_t)nr * nth, hplane = (uint32_t)(nr - 1) * nth;
    const T hdt = from_words<T>(I.hdt), dt = from_words<T>(I.dt);
    const int slot = lane_on ? g * nth + j : j;          // idle lanes never write
    const int gbase = lane_on ? g * nth : 0;

    // FP64 per-point mode: stage the block's radial rows in LDS
    const int bnA = max(wi.group * G * S, 1) - 1;
    const int bnB = min((wi.group * G + G) * S, nr - 1);
    double *lrow_f = lrows, *lrow_h = lrows + (size_t)(bnB - bnA + 1) * kRadRow;
    double cs_j = 0.0, s2_j = 0.0;
    if constexpr (W == 1 && ONFLY) {
        const int nf = (bnB - bnA + 1) * kRadRow, nh = (bnB - bnA) * kRadRow;
        const GLB double *rf = gptr(I.rf) + bnA * kRadRow, *rh = gptr(I.rh) + bnA * kRadRow;
        for (int q = threadIdx.x; q < nf + nh; q += NT) lrows[q] = q < nf ? rf[q] : rh[q - nf];
        if (lane_on) {
            cs_j = gptr(I.trig)[j];
            s2_j = gptr(I.trig)[nth + j];
        }
    }

    // double: this row's weights and reflected source rows in registers
    double wreg[2 * kMaxReach + 1];
    int qrow[2 * kMaxReach + 1];
    if constexpr (W == 1) {
#pragma unroll
        for (int k = 0; k < 2 * kMaxReach + 1; ++k) {
            const int kk = k - kMaxReach;
            const bool tap_on = lane_on && kk >= -R && kk <= R;
            wreg[k] = tap_on ? wtab[(uint32_t)((kk + R) * nth + j)] : 0.0;
            qrow[k] = tap_on ? tap_row(j, kk, nth) : 0;
        }
    }

    // zero radial boundary nodes owned by this segment
    const Pt<T> zero = {{mp_from<T>(0.0), mp_from<T>(0.0)}, {mp_from<T>(0.0), mp_from<T>(0.0)}};
    if (seg_on) {
        if (c0 == 0) gst_pt(uout, plane, (uint32_t)j, zero);
        if (c1 == nr) gst_pt(uout, plane, (uint32_t)((nr - 1) * nth + j), zero);
    }
    const int a = max(c0, 1) - 1;          // first node read
    const int e = min(c1, nr - 1);         // nodes a..e read; outputs a+1 .. e-1
    if constexpr (W == 4) {
        // quad-double: two exchanges per column (u^n, then the half step) with
        // the stages in sequence, which keeps fewer quad-double values live
        Pt<T> u_prev = zero, uh_prev = zero;
        cx<T> l_prev = zero.phi, lh_prev = zero.phi;
        Pt<T> u_next = (seg_on && a <= e) ? gld_pt<T>(uin, plane, (uint32_t)(a * nth + j)) : zero;
        d2 *xp = &xb[0][0][0][0], *xh = &xb[0][1][0][0];
        for (int t = 0; t < S + 2; ++t) {
            const int col = a + t;
            const Pt<T> u_cur = u_next;
            if (seg_on && col + 1 <= e) u_next = gld_pt<T>(uin, plane, (uint32_t)((col + 1) * nth + j));
            if (lane_on) xput<T>(xp, NT, slot, u_cur.phi);
            __syncthreads();
            const cx<T> l_cur = theta_stencil<T>(xp + gbase, NT, j, nth, R, wtab, wreg, qrow);
            // (lw1) at half node col-1/2 (index col-1)
            const bool h_on = seg_on && col <= e && t >= 1;
            T cf[8];
            load_coef<T>(gptr(I.ch), hplane, (uint32_t)(min(max(col - 1, 0), nr - 2) * nth + j), cf);
            const Pt<T> bar = pt_avg(u_prev, u_cur);
            const Pt<T> uh_cur = lw_stage(bar, bar, pt_diff(u_prev, u_cur), c_avg(l_prev, l_cur), cf, hdt);
            if (lane_on) xput<T>(xh, NT, slot, uh_cur.phi);
            __syncthreads();
            const cx<T> lh_cur = theta_stencil<T>(xh + gbase, NT, j, nth, R, wtab, wreg, qrow);
            if (h_on && t >= 2) {
                // (lw2) at node col-1
                const int i = col - 1;
                load_coef<T>(gptr(I.cf), plane, (uint32_t)(i * nth + j), cf);
                const Pt<T> un = lw_stage(u_prev, pt_avg(uh_prev, uh_cur), pt_diff(uh_prev, uh_cur),
                                          c_avg(lh_prev, lh_cur), cf, dt);
                gst_pt(uout, plane, (uint32_t)(i * nth + j), un);
            }
            u_prev = u_cur;
            l_prev = l_cur;
            uh_prev = uh_cur;
            lh_prev = lh_cur;
        }
        return;
    }
    Pt<T> u_m2 = zero, u_m1 = zero;        // u^n at c-2, c-1
    Pt<T> uh_m52 = zero, uh_m32 = zero;    // half-step values at c-5/2, c-3/2
    cx<T> l_m1 = zero.phi, lh_m52 = zero.phi;
    // one column: exchange, stencils, stage 2 at c-2, stage 1 at c-1/2
    auto column = [&](int k, const Pt<T> &u_c) {
        const int c = a + k;
        d2 *xp = &xb[k & 1][0][0][0], *xh = &xb[k & 1][1][0][0];
        if (lane_on) {
            xput<T>(xp, NT, slot, u_c.phi);
            xput<T>(xh, NT, slot, uh_m32.phi);
        }
        __syncthreads();
        const cx<T> l_c = theta_stencil<T>(xp + gbase, NT, j, nth, R, wtab, wreg, qrow);
        const cx<T> lh_m32 = theta_stencil<T>(xh + gbase, NT, j, nth, R, wtab, wreg, qrow);
        if (k >= 3) {
            // (lw2) at node c-2; indices are clamped so inactive lanes read valid memory
            const int i = c - 2;
            const bool on = seg_on && i <= e - 1;
            const int ic = min(max(i, 1), nr - 2);
            const Pt<T> un = stage_at<T, ONFLY>(gptr(I.cf), lrow_f + min(max(i - bnA, 0), bnB - bnA) * kRadRow, plane,
                                                (uint32_t)(ic * nth + j), cs_j, s2_j, u_m2, pt_avg(uh_m52, uh_m32),
                                                pt_diff(uh_m52, uh_m32), c_avg(lh_m52, lh_m32), dt);
            if (on) gst_pt(uout, plane, (uint32_t)(i * nth + j), un);
        }
        Pt<T> uh_new = zero;
        if (k >= 1) {
            // (lw1) at half node c-1/2 (index c-1)
            const int hc = min(max(c - 1, 0), nr - 2);
            const Pt<T> bar = pt_avg(u_m1, u_c);
            uh_new = stage_at<T, ONFLY>(gptr(I.ch), lrow_h + min(max(c - 1 - bnA, 0), bnB - bnA - 1) * kRadRow,
                                        hplane, (uint32_t)(hc * nth + j), cs_j, s2_j, bar, bar, pt_diff(u_m1, u_c),
                                        c_avg(l_m1, l_c), hdt);
        }
        u_m2 = u_m1;
        u_m1 = u_c;
        l_m1 = l_c;
        uh_m52 = uh_m32;
        lh_m52 = lh_m32;
        uh_m32 = uh_new;
    };
    if constexpr (SEG > 0) {
        Pt<T> ucol[SEG + 2];
#pragma unroll
        for (int q = 0; q < SEG + 2; ++q)
            ucol[q] = (seg_on && a + q <= e) ? gld_pt<T>(uin, plane, (uint32_t)((a + q) * nth + j)) : zero;
#pragma unroll
        for (int k = 0; k < SEG + 3; ++k) column(k, k < SEG + 2 ? ucol[k] : zero);
    } else {
        Pt<T> u_next = (seg_on && a <= e) ? gld_pt<T>(uin, plane, (uint32_t)(a * nth + j)) : zero;
        for (int k = 0; k < S + 3; ++k) {
            const Pt<T> u_c = u_next;
            if (seg_on && a + k + 1 <= e) u_next = gld_pt<T>(uin, plane, (uint32_t)((a + k + 1) * nth + j));
            column(k, u_c);
        }
    }
}

// Segment taken by block b of an n-block launch of one instance: the GPU deals
// block b to XCD b mod 8; the blocks one XCD receives take consecutive
// segments (XCD x owns the contiguous range after those of XCDs 0..x-1).
MPA int xcd_segment(int b, int n) {
    const int x = b % 8, r = b / 8, q = n / 8, rem = n % 8;
    return x * q + min(x, rem) + r;
}

// ------------------------------------------------------------------ wide sweep
// The G = NT / n_theta groups of a block take the columns of one r* segment
// in turn, each lane a run of P consecutive columns of its theta row: in
// iteration t group g handles the run kb = tG + g, columns kb P .. kb P + P-1
// of the nodes a..e the segment reads.  Every column of the segment is
// computed once (only the segment's two edge columns are shared with its
// neighbours); inside a run the left neighbour is in registers, across runs
// it comes through LDS (u^n and L(Phi^n) for stage 1, the half step and its L
// for stage 2).  P > 1 gives each lane independent chains to interleave.
//
// Exchange arrays are circular over G + 1 run slots (run kb in slot
// kb mod (G+1)).  Phi and the half-step Phi of all P columns carry reflected
// ghost rows (n_theta + 2 kMaxReach rows, row q at position q + kMaxReach,
// holding the raw value of the row it mirrors: the ghost sign is in the
// weights), so a stencil reads 2 kMaxReach + 1 consecutive rows; Pi, L(Phi)
// and the half-step Pi and L are kept for the last column of a run only.
// Per iteration (three barriers):
//   put Phi^n (P columns), Pi^n of the last                  | B1
//   stage 2 at the nodes left of each column of the previous iteration's
//     run kb - G (its left neighbour run kb - G - 1 sits in slot
//     (kb - G - 1) mod (G+1) == kb mod (G+1), the slot of this iteration);
//   L(Phi^n) of the P columns, put the last; read u^n left of the run | B2
//   read L left of the run; stage 1 at the P half nodes left of the
//     columns; put them                                      | B3
//   L of the half steps, put the last.
// Slot kb mod (G+1) is next rewritten in the following iteration by group
// g + 1 (or two iterations on by group 0); every read of a slot precedes
// that rewrite by at least one barrier.
MPA int wide_groups(int nt, int nth) { return nt / nth; }

// LDS bytes of the exchange arrays of the wide kernel with runs of p columns
template <class T> MPA size_t wide_xchg_bytes(int nt, int nth, int p) {
    constexpr int CH = words_of<T>::value == 1 ? 1 : words_of<T>::value;
    const int D = wide_groups(nt, nth) + 1, RS = nth + 2 * kMaxReach;
    return (size_t)D * CH * sizeof(d2) * (2 * (size_t)p * RS + 4 * (size_t)nth);
}
// LDS bytes of the FP64 per-point radial rows of a segment of `segcols` outputs
MPA size_t wide_rows_bytes(int segcols) { return (size_t)(2 * segcols + 3) * kRadRow * sizeof(double); }

template <class T>
__device__ __forceinline__ void xput_ghosted(d2 *slot, int rs, int j, int nth, const cx<T> &v) {
    xput<T>(slot, rs, kMaxReach + j, v);
    if (j < kMaxReach) xput<T>(slot, rs, kMaxReach - 1 - j, v);
    if (j >= nth - kMaxReach) xput<T>(slot, rs, kMaxReach + 2 * nth - 1 - j, v);
}

// angular operator at row j from a ghosted slot (see theta_stencil).
// wmp: double-double weights of row j held in registers (taps -kMaxReach ..
// kMaxReach, zero beyond the reach), or nullptr to load them per tap.
template <class T>
__device__ __forceinline__ cx<T> stencil_ghosted(const d2 *slot, int rs, int j, int nth, int reach,
                                                 const GLB double *__restrict__ wt, const double *w,
                                                 const T *wmp = nullptr) {
    constexpr int W = words_of<T>::value;
    Acc<T> re, im;
    if (W == 2 && wmp) {
        // all eleven taps, in order; taps beyond the reach have weight 0 and
        // read a valid ghosted row, their exact zero products change nothing
#pragma unroll
        for (int k = 0; k < 2 * kMaxReach + 1; ++k) {
            const cx<T> x = xget<T>(slot, rs, j + k);      // row j + k - kMaxReach
            re.prod(wmp[k], x.re);
            im.prod(wmp[k], x.im);
        }
    } else if constexpr (W == 1) {
#pragma unroll
        for (int k = 0; k < 2 * kMaxReach + 1; ++k) {
            const cx<T> x = xget<T>(slot, rs, j + k);      // row j + k - kMaxReach
            re.prod(w[k], x.re);
            im.prod(w[k], x.im);
        }
    } else if constexpr (W == 2) {
        // double-double: the weight (a global load) and the LDS value of tap
        // k + 1 are requested before tap k is accumulated, so a tap's loads
        // are in flight during the previous tap's arithmetic (same operations
        // in the same order as the plain loop)
        const GLB double *wrow = wt + (uint32_t)j;
        cx<T> x = xget<T>(slot, rs, kMaxReach + j - reach);
        T wk = gld<T>(wrow, (uint32_t)nth, 0u);
#pragma unroll 1
        for (int k = -reach; k <= reach; ++k) {
            const bool more = k < reach;
            const int kn = more ? k + 1 : k;
            const cx<T> xn = xget<T>(slot, rs, kMaxReach + j + kn);
            const T wn = gld<T>(wrow + (uint32_t)((kn + reach) * W * nth), (uint32_t)nth, 0u);
            re.prod(wk, x.re);
            im.prod(wk, x.im);
            x = xn;
            wk = wn;
        }
    } else {
        // quad-double: the weight of tap k + 1 (a global load) is requested
        // before tap k is accumulated; its LDS value is read in the tap itself
        const GLB double *wrow = wt + (uint32_t)j;
        T wk = gld<T>(wrow, (uint32_t)nth, 0u);
#pragma unroll 1
        for (int k = -reach; k <= reach; ++k) {
            const int kn = k < reach ? k + 1 : k;
            const T wn = gld<T>(wrow + (uint32_t)((kn + reach) * W * nth), (uint32_t)nth, 0u);
            const cx<T> x = xget<T>(slot, rs, kMaxReach + j + k);
            re.prod(wk, x.re);
            im.prod(wk, x.im);
            wk = wn;
        }
    }
    return {re.result(), im.result()};
}

// CM: coefficient mode -- 0 stored planes, 1 (FP64) per point from radial
// rows staged in LDS, 2 (FP64, n_theta a multiple of the wavefront size, so
// a wavefront lies in one group and its column is uniform) per point from
// radial rows read with scalar loads, 3 (multiword) stored planes requested
// one phase ahead: the planes of the next iteration's two stages are loaded
// right after this iteration's stage 1, so their memory latency overlaps
// the half-step stencil, the next puts and the first barrier instead of
// following a barrier.  Same values, same arithmetic: bitwise equal to 0.
// 4 (double-double) per point from double-double radial rows (the FP64
// mode's factors, coef_dd_point): no coefficient planes are read; the
// coefficients differ from the stored planes by rounding only.
// Launch arguments of a one-instance launch, passed by value so that the
// state loads need no descriptor load first (they arrive with the kernel
// arguments, preloaded into SGPRs where the hardware supports it).
struct WideArgs {
    const double *uin;
    double *uout;
    int nr, nth, segcols, blocks;
};

// TM > 0: at most TM iterations (the host checks), all loads issued up front.
// ONE: a one-instance launch (items unused, geometry and state pointers from
// wa; the blocks take the segments in the XCD-aware order of the host's
// xcd_order); otherwise every block reads its work item and descriptor.
// NS > 1 (with TM > 0): NS steps per launch.  The block reads NS columns on
// each side of its segment; after every step the stage-2 results stay in the
// lanes' registers (shifted one node left: a lane's stage 2 is at the node left
// of its column) and the valid range shrinks by one column at each side that
// is not a domain boundary.  At the right domain boundary NS extra columns
// carry node n_r - 1 as it shifts; boundary nodes are reset to zero each step.
template <class T, int NT, int P, int CM, int TM, bool ONE, int NS>
__global__ __launch_bounds__(NT) void lw_wide_kernel(const double *wa_uin, double *wa_uout, int wa_nr, int wa_nth,
                                                     int wa_segcols, int wa_blocks,
                                                     const InstDev *__restrict__ insts,
                                                     const WorkItem *__restrict__ items, int parity) {
    constexpr int W = words_of<T>::value;
    constexpr int CH = W == 1 ? 1 : W;
    constexpr int RM = kMaxReach;
    static_assert(NS == 1 || TM > 0, "fused steps need the unrolled form");
    extern __shared__ d2 xs[];
    // (the one-instance arguments are plain scalars, first in the list, so
    // the hardware can preload them into SGPRs)
    const WideArgs wa{wa_uin, wa_uout, wa_nr, wa_nth, wa_segcols, wa_blocks};
    const WorkItem wi = ONE ? WorkItem{0, xcd_segment(blockIdx.x, wa.blocks)} : items[blockIdx.x];
    const InstDev &I = insts[wi.inst];
    const int nr = ONE ? wa.nr : I.nr, nth = ONE ? wa.nth : I.nth, B = ONE ? wa.segcols : I.segcols;
    const int R = I.reach;
    const int G = wide_groups(NT, nth), D = G + 1, RS = nth + 2 * RM;
    const int g = threadIdx.x / nth, j = threadIdx.x - g * nth;
    const bool lane_on = g < G;
    const int c0 = wi.group * B, c1 = min(c0 + B, nr);
    const int a = max(c0 - NS, 0), e = min(c1 - 1 + NS, nr - 1);
    const int KR = e - a + 1;                       // columns a..e (nodes that exist)
    const int K = KR + ((NS > 1 && e == nr - 1) ? NS : 0);
    const int SP = P * CH * RS;                     // doubles-pairs per ghosted slot
    d2 *const XP = xs;                              // Phi^n        [slot][p][chunk][RS]
    d2 *const XH = XP + D * SP;                     // half-step Phi
    d2 *const XPI = XH + D * SP;                    // Pi^n, last column   [slot][chunk][nth]
    d2 *const XHI = XPI + D * CH * nth;             // half-step Pi, last column
    d2 *const XL = XHI + D * CH * nth;              // L(Phi^n), last column
    d2 *const XLH = XL + D * CH * nth;              // L(half-step Phi), last column
    double *const lrow_f = (double *)(XLH + D * CH * nth);    // FP64 per-point: radial rows, nodes a..e
    double *const lrow_h = lrow_f + KR * kRadRow;             //                 half nodes a..e-1
    const GLB double *uin = gptr(ONE ? wa.uin : (const double *)I.u[parity]);
    GLB double *uout = gptr(ONE ? wa.uout : I.u[parity ^ 1]);
    const GLB double *wtab = gptr(I.wt);
    const uint32_t plane = (uint32_t)nr * nth, hplane = (uint32_t)(nr - 1) * nth;
    const int jj = lane_on ? j : 0;
    // the run's columns, requested before anything that needs the descriptor
    const int TI = (K + G * P - 1) / (G * P);       // iterations with columns (TM >= TI when TM > 0)
    Pt<T> ua[TM > 0 ? TM : 1][P];
    if constexpr (TM > 0) {
#pragma unroll
        for (int t = 0; t < TM; ++t)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int k = g * P + t * G * P + p;
                ua[t][p] = (lane_on && t < TI && k < KR) ? gld_pt<T>(uin, plane, (uint32_t)((a + k) * nth + j))
                                                        : Pt<T>{};
            }
    }
    const T hdt = from_words<T>(I.hdt), dt = from_words<T>(I.dt);

    double cs_j = 0.0, s2_j = 0.0;
    if constexpr (W == 1 && CM == 1) {
        const int nf = KR * kRadRow, nh = (KR - 1) * kRadRow;
        const GLB double *rf = gptr(I.rf) + a * kRadRow, *rh = gptr(I.rh) + a * kRadRow;
        for (int q = threadIdx.x; q < nf + nh; q += NT) lrow_f[q] = q < nf ? rf[q] : rh[q - nf];
    }
    if constexpr (W == 1 && CM > 0) {
        cs_j = gptr(I.trig)[jj];
        s2_j = gptr(I.trig)[nth + jj];
    }
    T cs_m = mp_from<T>(0.0), s2_m = mp_from<T>(0.0);    // multiword per-point mode: cos, sin^2 of row j
    if constexpr (W == 2 && CM == 4) {
        cs_m = gld<T>(gptr(I.trig), (uint32_t)nth, (uint32_t)jj);
        s2_m = gld<T>(gptr(I.trig) + W * nth, (uint32_t)nth, (uint32_t)jj);
    }
    // one stage at node (half = false) or half node i, row j, with the
    // coefficients of that point
    // CM == 3: the planes of one stage's P points, loaded ahead of use
    auto load_planes = [&](bool half, int i, T *cf) {
        const GLB double *pl = gptr(half ? I.ch : I.cf);
        const uint32_t pn = half ? hplane : plane;
#pragma unroll
        for (int q = 0; q < 8; ++q) cf[q] = gld<T>(pl + q * W * pn, pn, (uint32_t)(i * nth + jj));
    };
    T pre2[CM == 3 ? P : 1][8], pre1[CM == 3 ? P : 1][8];
    auto stage = [&](bool half, int i, const Pt<T> &base, const Pt<T> &bar, const Pt<T> &d, const cx<T> &lbar,
                     const T &s, const T *pre) -> Pt<T> {
        if constexpr (CM == 3) {
            return lw_stage(base, bar, d, lbar, pre, s);
        } else if constexpr (W == 2 && CM == 4) {
            T c[8];
            coef_dd_point(gptr(half ? I.rh : I.rf) + (uint32_t)(i * kRadRow * W), cs_m, s2_m, c);
            return lw_stage(base, bar, d, lbar, c, s);
        } else if constexpr (W == 1 && CM == 2) {
            const int iu = __builtin_amdgcn_readfirstlane(i);
            return lw_stage_row(base, bar, d, lbar, (const CNS double *)(half ? I.rh : I.rf) + iu * kRadRow, cs_j,
                                s2_j, s);
        } else if constexpr (W == 1 && CM == 1) {
            return lw_stage_row(base, bar, d, lbar, (half ? lrow_h : lrow_f) + (i - a) * kRadRow, cs_j, s2_j, s);
        } else {
            const GLB double *pl = gptr(half ? I.ch : I.cf);
            const uint32_t pn = half ? hplane : plane;
            T cf[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) cf[q] = gld<T>(pl + q * W * pn, pn, (uint32_t)(i * nth + jj));
            return lw_stage(base, bar, d, lbar, cf, s);
        }
    };
    double wreg[2 * RM + 1];
    if constexpr (W == 1) {
#pragma unroll
        for (int k = 0; k < 2 * RM + 1; ++k) {
            const int kk = k - RM;
            wreg[k] = (lane_on && kk >= -R && kk <= R) ? wtab[(uint32_t)((kk + R) * nth + j)] : 0.0;
        }
    }
    // double-double forms that run two wavefronts per SIMD with or without them
    // (the loop form, and two unrolled iterations with fused steps): the row's
    // eleven weights in registers for the whole launch instead of one global
    // load per tap and stencil.  The forms at three wavefronts per SIMD keep the
    // loads (the 44 extra VGPRs would cost them a wavefront).
    constexpr bool WMP = W == 2 && (TM == 0 || (TM == 2 && NS > 1));
    T wmp[WMP ? 2 * RM + 1 : 1];
    if constexpr (WMP) {
#pragma unroll
        for (int k = 0; k < 2 * RM + 1; ++k) {
            const int kk = k - RM;
            wmp[k] = (kk >= -R && kk <= R) ? gld<T>(wtab + (uint32_t)((kk + R) * W * nth), (uint32_t)nth, (uint32_t)jj)
                                           : mp_from<T>(0.0);
        }
    }
    const Pt<T> zero = {{mp_from<T>(0.0), mp_from<T>(0.0)}, {mp_from<T>(0.0), mp_from<T>(0.0)}};
    if (lane_on && g == 0) {
        if (c0 == 0) gst_pt(uout, plane, (uint32_t)j, zero);
        if (c1 == nr) gst_pt(uout, plane, (uint32_t)((nr - 1) * nth + j), zero);
    }

    int k0 = g * P, sk = lane_on ? g : 0;           // first column of this lane's run and the run's slot
    // the slot's offsets into the ghosted arrays (sk * SP) and the per-row
    // arrays (sk * SN), stepped along with sk instead of multiplied out
    const int SN = CH * nth, GSP = G * SP, GSN = G * SN;
    int so = sk * SP, sn = sk * SN;
    Pt<T> u_l[P], uh_l[P];                          // stage-2 operands kept from the previous iteration:
    cx<T> lh_l[P];                                  // u^n left of each column, half steps, their L
#pragma unroll
    for (int p = 0; p < P; ++p) {
        u_l[p] = zero;
        uh_l[p] = zero;
        lh_l[p] = zero.phi;
    }
    // iteration t on the run's columns u_c; false once the last stage 2 is done
    int as = a;                                     // node of column 0 in the current step
    // iteration t on the run's columns u_c; stage 2 of the previous run goes to
    // global memory in the last step, else (fused steps) to u_out
    auto iteration = [&](int t, const Pt<T> *u_c, Pt<T> *u_out, bool last) -> bool {
        const int sl = sk == 0 ? G : sk - 1;        // slot of the run to the left
        const int slo = sk == 0 ? GSP : so - SP, sln = sk == 0 ? GSN : sn - SN;
        d2 *const xp = XP + so, *const xh = XH + so;
#pragma unroll
        for (int p = 0; p < P; ++p)
            if (lane_on && k0 + p < K) xput_ghosted<T>(xp + p * CH * RS, RS, j, nth, u_c[p].phi);
        const bool last_on = lane_on && k0 + P - 1 < K;
        if (last_on) xput<T>(XPI + sn, nth, j, u_c[P - 1].pi);
        __syncthreads();                                                        // B1
        // FP64 stages run on every lane with clamped indices (results of idle
        // lanes and of columns outside the segment are discarded); only the
        // stores are conditional, which keeps each phase one basic block.
        if constexpr (CM == 3) {
            if (t == 0) {
                // first iteration of a step: this iteration's stage-1 planes
                // (it has no stage 2)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    load_planes(true, min(max((NS == 1 ? a : as) + k0 + p - 1, a), e - 1), pre1[p]);
            }
        }
        if (t >= 1) {
            // stage 2 (lw2) at node a + kp - 1 for the columns kp of the previous run
            const int k0p = k0 - G * P;
            Pt<T> uh_m;                             // half step left of that run
            uh_m.phi = xget<T>(xh + (P - 1) * CH * RS, RS, RM + jj);
            uh_m.pi = xget<T>(XHI + sn, nth, jj);
            const cx<T> lh_m = xget<T>(XLH + sn, nth, jj);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int kp = k0p + p, i = (NS == 1 ? a : as) + kp - 1;
                const bool on = lane_on && kp >= 2 && kp < K;
                // (FP64 computes on every lane; the multiword types skip whole
                // wavefronts with nothing to do, which saves far more there)
                Pt<T> un = zero;
                if (W == 1 || on) {
                    const int ic = min(max(i, a), e);
                    const Pt<T> &ua = p == 0 ? uh_m : uh_l[p > 0 ? p - 1 : 0];
                    const cx<T> &la = p == 0 ? lh_m : lh_l[p > 0 ? p - 1 : 0];
                    un = stage(false, ic, u_l[p], pt_avg(ua, uh_l[p]), pt_diff(ua, uh_l[p]), c_avg(la, lh_l[p]), dt,
                               pre2[CM == 3 ? p : 0]);
                }
                if constexpr (NS == 1) {
                    if (on) gst_pt(uout, plane, (uint32_t)(i * nth + j), un);
                } else if (last) {
                    // nodes of the segment, radial boundary excluded
                    if (lane_on && i >= max(c0, 1) && i < min(c1, nr - 1)) gst_pt(uout, plane, (uint32_t)(i * nth + j), un);
                } else {
                    u_out[p] = (i == 0 || i == nr - 1) ? zero : un;
                }
            }
        }
        if (t == TI) return false;
        cx<T> l_c[P];
#pragma unroll
        for (int p = 0; p < P; ++p)
            l_c[p] = stencil_ghosted<T>(xp + p * CH * RS, RS, jj, nth, R, wtab, wreg, WMP ? wmp : nullptr);
        if (last_on) xput<T>(XL + sn, nth, j, l_c[P - 1]);
        Pt<T> u_m1;                                 // u^n left of the run
        u_m1.phi = xget<T>(XP + slo + (P - 1) * CH * RS, RS, RM + jj);
        u_m1.pi = xget<T>(XPI + sln, nth, jj);
        __syncthreads();                                                        // B2
        Pt<T> uh[P];
        {
            const cx<T> l_m1 = xget<T>(XL + sln, nth, jj);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                // stage 1 (lw1) at half node a + k - 1/2 (half index a + k - 1)
                const int k = k0 + p, h = (NS == 1 ? a : as) + k - 1;
                const bool on = lane_on && k >= 1 && k < K;
                uh[p] = zero;
                if (W > 1 && !on) continue;
                const int hc = min(max(h, a), e - 1);
                const Pt<T> &ua = p == 0 ? u_m1 : u_c[p > 0 ? p - 1 : 0];
                const cx<T> &la = p == 0 ? l_m1 : l_c[p > 0 ? p - 1 : 0];
                const Pt<T> bar = pt_avg(ua, u_c[p]);
                uh[p] = stage(true, hc, bar, bar, pt_diff(ua, u_c[p]), c_avg(la, l_c[p]), hdt, pre1[CM == 3 ? p : 0]);
                if (on) xput_ghosted<T>(xh + p * CH * RS, RS, j, nth, uh[p].phi);
            }
            if (last_on && k0 + P - 1 >= 1) xput<T>(XHI + sn, nth, j, uh[P - 1].pi);
        }
        if constexpr (CM == 3) {
            // the next iteration's planes: its stage 2 takes this run's
            // columns, its stage 1 the next run's
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int base = (NS == 1 ? a : as) - 1;
                load_planes(false, min(max(base + k0 + p, a), e), pre2[p]);
                load_planes(true, min(max(base + k0 + G * P + p, a), e - 1), pre1[p]);
            }
        }
        __syncthreads();                                                        // B3
        cx<T> lh[P];
#pragma unroll
        for (int p = 0; p < P; ++p)
            lh[p] = stencil_ghosted<T>(xh + p * CH * RS, RS, jj, nth, R, wtab, wreg, WMP ? wmp : nullptr);
        if (last_on && k0 + P - 1 >= 1) xput<T>(XLH + sn, nth, j, lh[P - 1]);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            u_l[p] = p == 0 ? u_m1 : u_c[p > 0 ? p - 1 : 0];
            uh_l[p] = uh[p];
            lh_l[p] = lh[p];
        }
        k0 += G * P;
        sk = sl;                                    // (kb + G) mod (G+1) == (kb - 1) mod (G+1)
        so = slo;
        sn = sln;
        return true;
    };
    if constexpr (TM > 0) {
        // every column of the lane was requested up front (above): one memory
        // latency per launch instead of one per iteration
        if constexpr (NS == 1) {
#pragma unroll
            for (int t = 0; t <= TM; ++t)
                if (!iteration(t, ua[t < TM ? t : TM - 1], nullptr, true)) break;
        } else {
#pragma unroll
            for (int st = 0; st < NS; ++st) {
#pragma unroll
                for (int t = 0; t <= TM; ++t)
                    if (!iteration(t, ua[t < TM ? t : TM - 1], ua[t > 0 ? t - 1 : 0], st == NS - 1)) break;
                k0 = g * P;                         // next step: same lanes, same slots,
                sk = lane_on ? g : 0;               // columns one node further left
                so = sk * SP;
                sn = sk * SN;
                --as;
            }
        }
    } else {
        Pt<T> u_next[P];
#pragma unroll
        for (int p = 0; p < P; ++p)
            u_next[p] = (lane_on && k0 + p < K) ? gld_pt<T>(uin, plane, (uint32_t)((a + k0 + p) * nth + j)) : zero;
        for (int t = 0;; ++t) {
            Pt<T> u_c[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                u_c[p] = u_next[p];
                const int kn = k0 + G * P + p;
                if (lane_on && kn < K) u_next[p] = gld_pt<T>(uin, plane, (uint32_t)((a + kn) * nth + j));
            }
            if (!iteration(t, u_c, nullptr, true)) break;
        }
    }
}

// ------------------------------------------------------------------ slab sweep (persistent)
// One launch advances n steps of one FP64 instance with per-point
// coefficients.  Block b owns the r* segment xcd_segment(b, nseg) of B = G R
// nodes [c0, c0 + B) for the whole launch: group g (n_theta lanes, one per
// theta row) holds the R columns c0 + gR .. c0 + gR + R - 1 in registers, and
// Phi of every column also sits in LDS (with reflected ghost rows) for the
// angular stencil.  Only two values per row cross a segment edge per step,
// through global memory, each signalled by a per-wavefront flag holding the
// tag of the step it belongs to:
//   E1 (to the right neighbour): u^n and L(Phi^n) at the segment's last node,
//       the left operands of the neighbour's first half node;
//   E2 (to the left neighbour): the half step and its L at the segment's
//       first half node c0 - 1/2, the right operands of the neighbour's last
//       node.
// A step has four phases.  Phases 1 and 3 end with a block barrier: the next
// phase reads what the neighbouring groups wrote.  Phases 2 and 4 end with a
// sync of the group's own waves in FP64 and double-double: the stencil that
// follows reads only the group's columns (quad-double, short of LDS for the
// separate slots this needs, closes them with block barriers too):
//   1. L(Phi^n) of the lane's R columns to LDS (the group's last column
//      first: the last group stores it as E1 right away and sets the flag at
//      the end of the phase); Pi^n of that column to LDS.
//   2. Stage 1 at the R half nodes left of the columns.  The first takes u^n
//      and L left of the group from the group to the left, or for group 0
//      from E1 of the left neighbour (waiting for its flag, after the other
//      half nodes).  Half-step Phi to LDS.
//   3. L of the half steps to LDS (group 0 stores its first half node as E2
//      right away, flag at the end of the phase); half-step Pi of the group's
//      first half node to LDS.
//   4. Stage 2 at the R nodes.  The last takes the half step right of it from
//      the group to the right, or for the last group from E2 of the right
//      neighbour (waiting, after the other nodes).  Radial boundary nodes are
//      reset to zero; Phi^{n+1} to LDS.
// Each operand is the value the other sweeps use and every point takes the
// same operations in the same order, so the results are bitwise equal to
// theirs; no column is computed twice and no launch boundary falls between
// steps.  Exchange buffers alternate with the parity of the tag: a neighbour
// can rewrite a buffer two steps later only after it has waited for data this
// block produces after reading it.
//
// Every block must be resident at once: the host launches only after checking
// that the device holds them all (occupancy x compute units), and can launch
// cooperatively, which makes the runtime guarantee it.
// A wait polls at most `spin` times; a wave that gives up sets *err, every
// other wait whose flag has not arrived returns as soon as it sees *err, and
// the blocks leave the step
// loop after the next block barrier, so the kernel always ends; the host
// turns a nonzero *err into an error.  (A wait of phase 2 is checked after
// the barrier of phase 3, one of phase 4 after that of phase 1: a barrier
// lies between every check and the next wait that can set the flag, so all
// waves of a block leave at the same point.)
//
// Memory ordering across XCDs (each has its own L2) without cache-wide
// fences: every exchanged double and every flag is a relaxed atomic access
// at agent scope, which the hardware performs at the agent's coherence point
// (never from or into a non-coherent cached copy).  The producer waits for
// its data stores to complete (s_waitcnt) before it stores the flag; the
// consumer issues its data loads only after its flag load has returned the
// tag.  So the data a consumer reads are at least as new as the flag it saw.
// The agent-scope release and acquire fences would add an L2 write-back and
// an L2 invalidation per exchange: about 15 us per step on the 4096 x 128
// grid, measured, against 8.4 us for the whole step without them.
struct SlabArgs {
    const double *uin;
    double *uout;
    const double *rf, *rh, *trig, *wt;  // FP64 radial rows, theta factors; angular weights (all types)
    const double *ch, *cf;              // multiword: stored coefficient planes (half nodes, nodes)
    double *xbuf;                       // [2 parities][2: E1, E2][nseg][6 W][n_theta]
    unsigned long long *flags;          // [nseg][2: E1, E2][n_theta / 64], kSlabFlagPad apart
    int *err;
    long long base;                     // tag of the step before the launch's first
    long long spin;                     // polls before a wait gives up
    int nr, nth, nseg, reach, nsteps;
    double hdt[kMaxWords], dt[kMaxWords];   // dt / 2 and dt, W words
};
constexpr int kSlabFlagPad = 16;        // 128 bytes between flags

__device__ __forceinline__ unsigned long long *slab_flag(const SlabArgs &A, int seg, int dir, int wv) {
    return A.flags + ((size_t)(seg * 2 + dir) * (size_t)(A.nth >> 6) + (size_t)wv) * kSlabFlagPad;
}

// Wait (all lanes of a wavefront, same flag) until the flag holds `tag` or
// later.  false: *err was set, or `spin` polls passed (this wave then sets
// *err).  The flag is read first and the error word only while the flag is
// not there yet: a flag that has arrived costs one round trip to the
// coherence point, not two.  The signal fence keeps the compiler from moving
// the caller's data loads above the poll.
__device__ __forceinline__ bool slab_wait(unsigned long long *flag, unsigned long long tag, int *err, long long spin) {
    for (long long it = 0;; ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= tag) break;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (it >= spin) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return true;
}

__device__ __forceinline__ void slab_st(double *p, double v) {
    __hip_atomic_store((unsigned long long *)p, __builtin_bit_cast(unsigned long long, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double slab_ld(double *p) {
    return __builtin_bit_cast(double, __hip_atomic_load((unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <class T> __device__ __forceinline__ void slab_st_t(double *p, int nth, const T &v) {
#pragma unroll
    for (int w = 0; w < words_of<T>::value; ++w) slab_st(p + w * nth, mp_word(v, w));
}
template <class T> __device__ __forceinline__ T slab_ld_t(double *p, int nth) {
    T v;
#pragma unroll
    for (int w = 0; w < words_of<T>::value; ++w) mp_set_word(v, w, slab_ld(p + w * nth));
    return v;
}

// Store a row's six values (component-major, W words each, n_theta apart).
template <class T>
__device__ __forceinline__ void slab_put(double *dst, int nth, int j, const Pt<T> &u, const cx<T> &l) {
    constexpr int W = words_of<T>::value;
    slab_st_t(dst + (0 * W) * nth + j, nth, u.phi.re);
    slab_st_t(dst + (1 * W) * nth + j, nth, u.phi.im);
    slab_st_t(dst + (2 * W) * nth + j, nth, u.pi.re);
    slab_st_t(dst + (3 * W) * nth + j, nth, u.pi.im);
    slab_st_t(dst + (4 * W) * nth + j, nth, l.re);
    slab_st_t(dst + (5 * W) * nth + j, nth, l.im);
}
// After the wave's slab_put: wait until its stores have completed, then lane
// 0 sets the flag to `tag`.
__device__ __forceinline__ void slab_signal(unsigned long long *flag, unsigned long long tag, int j) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);      // every counter of the wave at zero: the stores have completed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if ((j & 63) == 0) __hip_atomic_store(flag, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
__device__ __forceinline__ void slab_take(double *src, int nth, int j, Pt<T> &u, cx<T> &l) {
    constexpr int W = words_of<T>::value;
    u.phi = {slab_ld_t<T>(src + (0 * W) * nth + j, nth), slab_ld_t<T>(src + (1 * W) * nth + j, nth)};
    u.pi = {slab_ld_t<T>(src + (2 * W) * nth + j, nth), slab_ld_t<T>(src + (3 * W) * nth + j, nth)};
    l = {slab_ld_t<T>(src + (4 * W) * nth + j, nth), slab_ld_t<T>(src + (5 * W) * nth + j, nth)};
}

// LDS bytes of the slab kernel for W words per real: Phi^n and half-step Phi
// of the B columns (ghosted), L of every column, Pi of one column per group; a
// complex value takes max(1, W) 16-byte chunks.  L(Phi^n) and the half
// step's L share one array.  With group-level syncs (W <= 2) it has one slot
// more per group, and Pi^n and the half-step Pi have arrays of their own;
// quad-double (block barriers only) shares those too.
MPA size_t slab_lds_bytes(int nt, int nth, int r, int words) {
    const int G = nt / nth, B = G * r, RS = nth + 2 * kMaxReach, CH = words == 1 ? 1 : words;
    if (words <= 2) return sizeof(d2) * CH * (2 * (size_t)B * RS + (size_t)(B + G) * nth + 2 * (size_t)G * nth);
    return sizeof(d2) * CH * (2 * (size_t)B * RS + (size_t)B * nth + (size_t)G * nth);
}

// NT threads = G groups of NTH (= n_theta, a multiple of 64) lanes; R
// columns per lane.  A lane keeps u^n and the half step of its R columns in
// registers; the angular operator of every column goes to LDS, where the lane
// and its neighbours read it back.  n_theta is a template parameter so that
// every LDS offset is an instruction immediate.  Coefficients: FP64 rebuilds
// them per point from radial rows (scalar loads); double-double loads the
// stored planes of its R columns once into registers (they do not change
// between steps) and keeps its angular weights in registers too; quad-double
// (at most two columns per lane) loads a stage's coefficients from the planes
// and each tap's weight, as the wide sweep does.
template <class T, int NT, int R, int NTH>
__global__ __launch_bounds__(NT) void lw_slab_kernel(SlabArgs A) {
    constexpr int RM = kMaxReach;
    constexpr int W = words_of<T>::value, CH = W == 1 ? 1 : W;
    static_assert(NT % NTH == 0 && NTH % 64 == 0, "groups of whole wavefronts");
    static_assert(W != 4 || R <= 2, "quad-double: at most two columns per lane");
    // DEC: phases 2 -> 3 and 4 -> 1 need only the group's own waves (see below)
    constexpr bool DEC = W <= 2;
    constexpr int nth = NTH, G = NT / nth, B = G * R, RS = nth + 2 * RM, WPG = NTH / 64;
    extern __shared__ d2 xs[];
    __shared__ int stop[2];                 // a wait gave up in phase 2, in phase 4
    __shared__ unsigned gcnt[G];            // group syncs passed, times the group's waves
    const int nr = A.nr;
    const int g = threadIdx.x / nth, j = threadIdx.x - g * nth, wv = j >> 6;
    const int seg = xcd_segment(blockIdx.x, A.nseg);
    const int c0 = seg * B, kg = g * R;
    const bool has_l = seg > 0, has_r = seg + 1 < A.nseg;
    // XL and XLH share their array; with block barriers only (quad-double)
    // so do EU and HU: phase 1 writes XL and EU, phase 2 reads them, phase 3
    // writes XLH and HU, phase 4 reads them, and a barrier separates each.
    // With group syncs after phases 2 and 4, a group can write while the
    // neighbouring groups still read, so what they read must not move: each
    // group has R + 1 slots of L, XLH of column r in slot r and XL in slot
    // r + 1 (the next group reads XL of the last column, the previous one
    // XLH of the first: neither is overwritten before the next block
    // barrier), and HU is apart from EU.
    d2 *const XP = xs;                  // Phi^n              [B][CH][RS]
    d2 *const XH = XP + B * CH * RS;    // half-step Phi      [B][CH][RS]
    d2 *const XL = XH + B * CH * RS;    // L(Phi^n)           [B or G (R + 1)][CH][nth]
    d2 *const XLH = XL;                 // L(half-step Phi)
    d2 *const EU = XL + (DEC ? B + G : B) * CH * nth;  // Pi^n of each group's last column  [G][CH][nth]
    d2 *const HU = DEC ? EU + G * CH * nth : EU;        // half-step Pi of each group's first half node
    auto sl_L = [](int k) { return DEC ? k + k / R + 1 : k; };     // slot of XL for column k
    auto sl_LH = [](int k) { return DEC ? k + k / R : k; };        // slot of XLH
    const uint32_t plane = (uint32_t)nr * nth, hplane = (uint32_t)(nr - 1) * nth;
    const GLB double *wtab = gptr(A.wt);
    const int reach = A.reach;
    const T hdt = from_words<T>(A.hdt), dt = from_words<T>(A.dt);
    double cs_j = 0.0, s2_j = 0.0;
    if constexpr (W == 1) {
        cs_j = gptr(A.trig)[j];
        s2_j = gptr(A.trig)[nth + j];
    }
    // angular weights of row j (taps -RM..RM, zero beyond the reach)
    // (quad-double loads each tap's weight in the stencil, as the wide sweep does)
    double wreg[2 * RM + 1];
    T wmp[W == 2 ? 2 * RM + 1 : 1];
#pragma unroll
    for (int k = 0; k < 2 * RM + 1; ++k) {
        const int kk = k - RM;
        const bool on = kk >= -reach && kk <= reach;
        if constexpr (W == 1)
            wreg[k] = on ? wtab[(uint32_t)((kk + reach) * nth + j)] : 0.0;
        else if constexpr (W == 2)
            wmp[k] = on ? gld<T>(wtab + (uint32_t)((kk + reach) * W * nth), (uint32_t)nth, (uint32_t)j) : mp_from<T>(0.0);
    }
    const T z = mp_from<T>(0.0);
    const Pt<T> zero = {{z, z}, {z, z}};
    // double-double: the coefficients of the lane's half nodes and nodes,
    // once (clamped indices where a node or half node does not exist; unused).
    // Quad-double loads a stage's eight from the planes when it needs them.
    T cfh[W == 2 ? R : 1][8], cff[W == 2 ? R : 1][8];
    auto load_cf = [&](bool half, int i, T *c) {
        const GLB double *pl = gptr(half ? A.ch : A.cf);
        const uint32_t pn = half ? hplane : plane;
#pragma unroll
        for (int q = 0; q < 8; ++q) c[q] = gld<T>(pl + q * W * pn, pn, (uint32_t)(i * nth + j));
    };
    if constexpr (W == 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t ih = (uint32_t)(min(max(c0 + kg + r - 1, 0), nr - 2) * nth + j);
            const uint32_t in = (uint32_t)(min(c0 + kg + r, nr - 1) * nth + j);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                cfh[r][q] = gld<T>(gptr(A.ch) + q * W * hplane, hplane, ih);
                cff[r][q] = gld<T>(gptr(A.cf) + q * W * plane, plane, in);
            }
        }
    }
    Pt<T> u[R];
    // Phi of the lane's columns (and below, of its half nodes) is in LDS for
    // the stencils.  FP64 and quad-double read it back there where a stage
    // needs it instead of keeping a second copy in registers for the whole
    // step (the same bits; fewer spills); double-double, which does not
    // spill, runs faster with the register copy.
    constexpr bool PL = W != 2;
    auto U = [&](int r) {
        Pt<T> v = u[r];
        if constexpr (PL) v.phi = xget<T>(XP + (kg + r) * CH * RS, RS, RM + j);
        return v;
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = c0 + kg + r;
        u[r] = i < nr ? gld_pt<T>(gptr(A.uin), plane, (uint32_t)(i * nth + j)) : zero;
        xput_ghosted<T>(XP + (kg + r) * CH * RS, RS, j, nth, u[r].phi);
    }
    // FP64: radial row of node (or half node) i, wave-uniform: scalar loads.
    // The row of a phase's stage r > 0 is requested only once stage r - 1 has
    // a result (`after`, through an empty asm): one 32-SGPR row is live at a
    // time instead of R, which the SGPR file cannot hold besides the launch
    // arguments (they would be parked in VGPR lanes and read back around
    // every use).
    auto row = [&](bool half, int i) {
        const int iu = __builtin_amdgcn_readfirstlane(i);
        return (const CNS double *)(half ? A.rh : A.rf) + iu * kRadRow;
    };
    auto row_after = [&](bool half, int i, double after) {
        int iu = __builtin_amdgcn_readfirstlane(i);
        asm volatile("" : "+s"(iu) : "v"(after));
        return (const CNS double *)(half ? A.rh : A.rf) + iu * kRadRow;
    };
    // The neighbour exchanges chain the blocks through their edge groups (the
    // last group's E1, the first group's E2); the other groups have slack.
    // In FP64 (four wavefronts per SIMD) the edge groups' waves issue first:
    // the step shortens by about 6 %.  (Double-double, one wavefront per
    // SIMD in its tuned shape, ran slower with it; quad-double did not change.)
    if constexpr (W == 1) {
        if (g == 0 || g == G - 1) __builtin_amdgcn_s_setprio(2);
    }
    if (threadIdx.x == 0) stop[0] = stop[1] = 0;
    if (threadIdx.x < G) gcnt[threadIdx.x] = 0;
    __syncthreads();
    // Sync of the group's waves: LDS writes before it are seen by the group's
    // reads after it.  One wave: program order (LDS keeps a wave's accesses in
    // order; the fences keep the compiler's).  Several: a counter in LDS,
    // polled at most `spin` times (a wave that gives up sets *err and stop[i]).
    unsigned gk = 0;
    auto group_sync = [&](int i) {
        if constexpr (WPG == 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            gk += WPG;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if ((j & 63) == 0) __hip_atomic_fetch_add(&gcnt[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (long long it = 0; __hip_atomic_load(&gcnt[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < gk; ++it) {
                if (it >= A.spin) {
                    __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    stop[i] = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
    };
    for (int s = 0; s < A.nsteps; ++s) {
        const unsigned long long tag = (unsigned long long)(A.base + s + 1);
        const size_t xo = (size_t)(tag & 1) * 2 * A.nseg * 6 * W * nth;
        double *const x1 = A.xbuf + xo, *const x2 = A.xbuf + xo + (size_t)A.nseg * 6 * W * nth;
        // 1. L(Phi^n) to LDS, the group's last column first (the last group
        //    publishes it as E1 before the other columns); Pi^n of that column
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = R - 1 - q;
            const cx<T> l = stencil_ghosted<T>(XP + (kg + r) * CH * RS, RS, j, nth, reach, wtab, wreg,
                                               W == 2 ? wmp : nullptr);
            xput<T>(XL + sl_L(kg + r) * CH * nth, nth, j, l);
            if (q == 0 && g == G - 1 && has_r) slab_put(x1 + (size_t)seg * 6 * W * nth, nth, j, U(R - 1), l);
        }
        xput<T>(EU + g * CH * nth, nth, j, u[R - 1].pi);
        if (g == G - 1 && has_r) slab_signal(slab_flag(A, seg, 0, wv), tag, j);
        __syncthreads();
        if (DEC && stop[1]) break;
        // 2. stage 1 at the half nodes c0 + kg + r - 1/2 (half index c0 + kg + r - 1),
        //    r = 1..R-1 first: only r = 0 needs the values left of the group,
        //    which group 0 waits for (E1), so the wait follows the others
        Pt<T> uh[R];
        auto H = [&](int r) {
            Pt<T> v = uh[r];
            if constexpr (PL) v.phi = xget<T>(XH + (kg + r) * CH * RS, RS, RM + j);
            return v;
        };
        double prev1 = 0.0;                 // (orders the FP64 row loads, see row_after)
        auto stage1 = [&](int r, const Pt<T> &left, const cx<T> &ll) {
            // (half node -1/2 of the first segment and those past the right
            // boundary do not exist: computed with clamped rows, never used)
            const int k = kg + r, hc = min(max(c0 + k - 1, 0), nr - 2);
            const cx<T> lc = xget<T>(XL + sl_L(k) * CH * nth, nth, j);
            const Pt<T> ur = U(r);
            const Pt<T> bar = pt_avg(left, ur);
            if constexpr (W == 1) {
                const CNS double *rr = r == R - 1 && R > 1 ? row(true, hc) : row_after(true, hc, prev1);
                uh[r] = lw_stage_row(bar, bar, pt_diff(left, ur), c_avg(ll, lc), rr, cs_j, s2_j, hdt);
                prev1 = uh[r].pi.im;
            } else if constexpr (W == 2) {
                uh[r] = lw_stage(bar, bar, pt_diff(left, ur), c_avg(ll, lc), cfh[r], hdt);
            } else {
                T cf[8];
                load_cf(true, hc, cf);
                uh[r] = lw_stage(bar, bar, pt_diff(left, ur), c_avg(ll, lc), cf, hdt);
            }
            xput_ghosted<T>(XH + k * CH * RS, RS, j, nth, uh[r].phi);
        };
#pragma unroll
        for (int r = R - 1; r >= 1; --r) stage1(r, U(r - 1), xget<T>(XL + sl_L(kg + r - 1) * CH * nth, nth, j));
        {
            Pt<T> ua = zero;
            cx<T> la = zero.phi;
            if (g > 0) {
                ua.phi = xget<T>(XP + (kg - 1) * CH * RS, RS, RM + j);
                ua.pi = xget<T>(EU + (g - 1) * CH * nth, nth, j);
                la = xget<T>(XL + sl_L(kg - 1) * CH * nth, nth, j);
            } else if (has_l) {
                if (slab_wait(slab_flag(A, seg - 1, 0, wv), tag, A.err, A.spin))
                    slab_take(x1 + (size_t)(seg - 1) * 6 * W * nth, nth, j, ua, la);
                else
                    stop[0] = 1;
            }
            stage1(0, ua, la);
        }
        if constexpr (DEC) {
            group_sync(0);
        } else {
            __syncthreads();
            if (stop[0]) break;
        }
        // 3. L of the half steps to LDS, the group's first half node first
        //    (group 0 publishes it as E2 before the others); half-step Pi of it
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const cx<T> lh = stencil_ghosted<T>(XH + (kg + r) * CH * RS, RS, j, nth, reach, wtab, wreg,
                                                W == 2 ? wmp : nullptr);
            xput<T>(XLH + sl_LH(kg + r) * CH * nth, nth, j, lh);
            if (r == 0 && g == 0 && has_l) slab_put(x2 + (size_t)seg * 6 * W * nth, nth, j, H(0), lh);
        }
        xput<T>(HU + g * CH * nth, nth, j, uh[0].pi);
        if (g == 0 && has_l) slab_signal(slab_flag(A, seg, 1, wv), tag, j);
        __syncthreads();
        if (DEC && stop[0]) break;
        // 4. stage 2 at the nodes c0 + kg + r, r = 0..R-2 first: only r = R-1
        //    needs the half step right of the group, which the last group
        //    waits for (E2), so the wait follows the others
        double prev = 0.0;                  // (orders the FP64 row loads, see row_after)
        auto stage2 = [&](int r, const Pt<T> &right, const cx<T> &lr) {
            const int k = kg + r, i = c0 + k, ic = min(i, nr - 1);
            const cx<T> lc = xget<T>(XLH + sl_LH(k) * CH * nth, nth, j);
            const Pt<T> ur = U(r), hr = H(r);
            Pt<T> un;
            if constexpr (W == 1) {
                const CNS double *rr = r == 0 ? row(false, ic) : row_after(false, ic, prev);
                un = lw_stage_row(ur, pt_avg(hr, right), pt_diff(hr, right), c_avg(lc, lr), rr, cs_j, s2_j, dt);
                prev = un.pi.im;
            } else if constexpr (W == 2) {
                un = lw_stage(ur, pt_avg(hr, right), pt_diff(hr, right), c_avg(lc, lr), cff[r], dt);
            } else {
                T cf[8];
                load_cf(false, ic, cf);
                un = lw_stage(ur, pt_avg(hr, right), pt_diff(hr, right), c_avg(lc, lr), cf, dt);
            }
            u[r] = (i == 0 || i >= nr - 1) ? zero : un;
            xput_ghosted<T>(XP + k * CH * RS, RS, j, nth, u[r].phi);
        };
#pragma unroll
        for (int r = 0; r < R - 1; ++r) stage2(r, H(r + 1), xget<T>(XLH + sl_LH(kg + r + 1) * CH * nth, nth, j));
        {
            Pt<T> ub = zero;
            cx<T> lb = zero.phi;
            if (g < G - 1) {
                ub.phi = xget<T>(XH + (kg + R) * CH * RS, RS, RM + j);
                ub.pi = xget<T>(HU + (g + 1) * CH * nth, nth, j);
                lb = xget<T>(XLH + sl_LH(kg + R) * CH * nth, nth, j);
            } else if (has_r) {
                if (slab_wait(slab_flag(A, seg + 1, 1, wv), tag, A.err, A.spin))
                    slab_take(x2 + (size_t)(seg + 1) * 6 * W * nth, nth, j, ub, lb);
                else
                    stop[1] = 1;
            }
            stage2(R - 1, ub, lb);
        }
        if constexpr (DEC) {
            group_sync(1);
        } else {
            __syncthreads();
            if (stop[1]) break;
        }
    }
    // (with group syncs a wait of the last phase 4 is seen only after a barrier)
    if constexpr (DEC) __syncthreads();
    if (stop[0] | stop[1]) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = c0 + kg + r;
        if (i < nr) gst_pt(gptr(A.uout), plane, (uint32_t)(i * nth + j), U(r));
    }
}

}  // namespace lwk
