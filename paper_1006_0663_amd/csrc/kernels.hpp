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

// 1/sqrt(x), x > 0: correctly rounded float seed, two Newton steps in double
// (same basic operations on host and device, so both give the same bits)
MPA double rsqrt_nr(double x) {
    double y = (double)(1.0f / sqrtf((float)x));
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

MPA void coef_fp64_point(const double *rr, double cs, double s2, double *c) {
    const double X = fma(-rr[kA2D], s2, rr[kVp2]);
    const double rq = rsqrt_nr(X);
    const double q = rq * rq;
    const double b = rr[kVp] * rq;
    c[0] = rr[kSIVp] * rq;
    c[1] = rr[kSD] * q;
    c[2] = q * fma(s2 * q, rr[kSIT8], -fma(b, rr[kSIT1], rr[kSIT6]));
    c[3] = -q * fma(b, fma(rr[kSIT3], cs, rr[kSIT2]), rr[kSIT7]);
    c[4] = q * rr[kST1];
    c[5] = q * fma(rr[kST3], cs, rr[kST2]);
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

template <class T> MPA cx<T> c_avg(const cx<T> &a, const cx<T> &b) {
    return {mp_pow2(mp_add_fast(a.re, b.re), 0.5), mp_pow2(mp_add_fast(a.im, b.im), 0.5)};
}
template <class T> MPA cx<T> c_diff(const cx<T> &a, const cx<T> &b) {     // b - a
    return {mp_add_fast(b.re, mp_neg(a.re)), mp_add_fast(b.im, mp_neg(a.im))};
}
template <class T> MPA Pt<T> pt_avg(const Pt<T> &a, const Pt<T> &b) { return {c_avg(a.phi, b.phi), c_avg(a.pi, b.pi)}; }
template <class T> MPA Pt<T> pt_diff(const Pt<T> &a, const Pt<T> &b) { return {c_diff(a.phi, b.phi), c_diff(a.pi, b.pi)}; }

// Angular operator of the value v held by lane j of a group, via the LDS
// buffer buf.  Callers alternate strictly between two buffers, so the single
// barrier between the write and the reads also orders this write after every
// lane's reads of the same buffer two exchanges earlier.
template <class T>
__device__ __forceinline__ cx<T> theta_apply(cx<T> v, cx<T> *buf, int j, int nth, int reach,
                                             const double *__restrict__ wt, bool active) {
    constexpr int W = words_of<T>::value;
    if (active) buf[j] = v;
    __syncthreads();
    Acc<T> re, im;
    auto tap = [&](int k) {
        int q = j + k;
        q = q < 0 ? -1 - q : (q >= nth ? 2 * nth - 1 - q : q);
        const cx<T> x = buf[q];
        const T w = ld<T>(wt + (size_t)(k + reach) * W * nth, (size_t)nth, (size_t)j);
        re.prod(w, x.re);
        im.prod(w, x.im);
    };
    if constexpr (W == 1) {
        // double: unrolled, all loads issued together
#pragma unroll
        for (int k = -kMaxReach; k <= kMaxReach; ++k)
            if (k >= -reach && k <= reach) tap(k);
    } else {
        // multiword: a rolled loop keeps only one tap's operands live
#pragma unroll 1
        for (int k = -reach; k <= reach; ++k) tap(k);
    }
    return {re.result(), im.result()};
}

// eight coefficients of node/half node i at row j: from the stored planes, or
// (FP64 with onfly) rebuilt from the radial row and the row's cos, sin^2
template <class T>
__device__ __forceinline__ void load_coef(const InstDev &I, const double *planes, const double *rows,
                                          size_t plane, bool on, int i, int j, double cs, double s2, T *c) {
    constexpr int W = words_of<T>::value;
    if constexpr (W == 1) {
        if (I.onfly) {
            double cc[8];
            int ii = on ? i : 0;
            // with n_theta >= 64 the active lanes of a wavefront share one
            // column: make the row index uniform so the row is read with
            // scalar loads
            if (I.nth >= 64) ii = __builtin_amdgcn_readfirstlane(ii);
            coef_fp64_point(rows + (size_t)ii * kRadRow, cs, s2, cc);
#pragma unroll
            for (int q = 0; q < 8; ++q) c[q] = on ? cc[q] : 0.0;
            return;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
        c[q] = on ? ld<T>(planes + (size_t)q * W * plane, plane, (size_t)i * I.nth + j) : mp_from<T>(0.0);
}

template <class T, int NT>
__global__ __launch_bounds__(NT) void lw_step_kernel(const InstDev *__restrict__ insts,
                                                     const WorkItem *__restrict__ items, int parity) {
    constexpr int W = words_of<T>::value;
    __shared__ cx<T> lds[2][NT];
    const WorkItem wi = items[blockIdx.x];
    const InstDev &I = insts[wi.inst];
    const int nr = I.nr, nth = I.nth, R = I.reach, S = I.segcols;
    const int G = NT / nth;
    const int g = threadIdx.x / nth, j = threadIdx.x - g * nth;
    const bool lane_on = g < G;
    const int seg = wi.group * G + g;
    const int c0 = seg * S, c1 = min(c0 + S, nr);
    const bool seg_on = lane_on && c0 < nr;
    const double *uin = I.u[parity];
    double *uout = I.u[parity ^ 1];
    const size_t plane = (size_t)nr * nth, hplane = (size_t)(nr - 1) * nth;
    const T hdt = from_words<T>(I.hdt), dt = from_words<T>(I.dt);

    // angular weights of this row (wt + tap * W * nth); rows of idle lanes read row 0
    const double *wrow = I.wt;
    cx<T> *buf0 = &lds[0][lane_on ? g * nth : 0], *buf1 = &lds[1][lane_on ? g * nth : 0];

    // zero radial boundary nodes owned by this segment
    if (seg_on) {
        const Pt<T> z = {{mp_from<T>(0.0), mp_from<T>(0.0)}, {mp_from<T>(0.0), mp_from<T>(0.0)}};
        if (c0 == 0) st_pt(uout, plane, (size_t)j, z);
        if (c1 == nr) st_pt(uout, plane, (size_t)(nr - 1) * nth + j, z);
    }
    // theta factors of this row for the FP64 per-point coefficients
    double cs_j = 0.0, s2_j = 0.0;
    if (words_of<T>::value == 1 && I.onfly && lane_on) {
        cs_j = I.trig[j];
        s2_j = I.trig[nth + j];
    }
    const int a = max(c0, 1) - 1;          // first node read
    const int e = min(c1, nr - 1);         // interior outputs are nodes a+1 .. e-1
    const Pt<T> zero = {{mp_from<T>(0.0), mp_from<T>(0.0)}, {mp_from<T>(0.0), mp_from<T>(0.0)}};
    Pt<T> u_prev = zero, u_cur, uh_prev = zero, uh_cur;
    cx<T> l_prev = zero.phi, l_cur, lh_prev = zero.phi, lh_cur;
    // Every lane runs the same S + 2 iterations (the barriers in theta_apply
    // must be reached uniformly); work outside the segment is masked.
    // the next column's state is loaded one iteration ahead
    Pt<T> u_next = (seg_on && a <= e) ? ld_pt<T>(uin, plane, (size_t)a * nth + j) : zero;
    for (int t = 0; t < S + 2; ++t) {
        const int col = a + t;
        const bool col_on = seg_on && col <= e;
        u_cur = u_next;
        if (seg_on && col + 1 <= e) u_next = ld_pt<T>(uin, plane, (size_t)(col + 1) * nth + j);
        l_cur = theta_apply<T>(u_cur.phi, buf0, lane_on ? j : 0, nth, R, wrow, lane_on);
        // (lw1) at half node (col-1)+1/2
        const bool h_on = col_on && t >= 1;
        T c[8];
        load_coef<T>(I, I.ch, I.rh, hplane, h_on, col - 1, j, cs_j, s2_j, c);
        {
            const Pt<T> bar = pt_avg(u_prev, u_cur);
            const Pt<T> d = pt_diff(u_prev, u_cur);
            const cx<T> lbar = c_avg(l_prev, l_cur);
            uh_cur = lw_stage(bar, bar, d, lbar, c, hdt);
        }
        lh_cur = theta_apply<T>(uh_cur.phi, buf1, lane_on ? j : 0, nth, R, wrow, lane_on);
        if (h_on && t >= 2) {
            // (lw2) at node col-1
            const int i = col - 1;
            load_coef<T>(I, I.cf, I.rf, plane, true, i, j, cs_j, s2_j, c);
            const Pt<T> barh = pt_avg(uh_prev, uh_cur);
            const Pt<T> dh = pt_diff(uh_prev, uh_cur);
            const cx<T> lbarh = c_avg(lh_prev, lh_cur);
            const Pt<T> un = lw_stage(u_prev, barh, dh, lbarh, c, dt);
            st_pt(uout, plane, (size_t)i * nth + j, un);
        }
        uh_prev = uh_cur;
        lh_prev = lh_cur;
        u_prev = u_cur;
        l_prev = l_cur;
    }
}

}  // namespace lwk
