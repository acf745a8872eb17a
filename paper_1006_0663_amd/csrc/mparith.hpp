// Multiword floating-point arithmetic on native FP64: double (1 word),
// double-double (2 words, ~106-bit significand) and quad-double (4 words,
// ~212-bit significand).  The paper evaluates its stencil in these three
// precisions, obtaining the wider ones from a library that represents a
// number as an unevaluated sum of doubles (Sec. "High-Order and
// High-Precision").  This header is a fresh implementation for gfx950 built
// only from error-free transforms:
//
//   two_sum       Knuth's branch-free exact sum  s + e = a + b
//   fast_two_sum  Dekker's exact sum, valid when |a| >= |b| (or a == 0)
//   two_prod      exact product p + e = a * b using one FMA
//
// double-double: addition is Joldes-Muller-Popescu (2017) AccurateDWPlusDW
// (relative error <= 3u^2), multiplication DWTimesDW3 and DWTimesFP3 (FMA
// based, <= 4u^2 and <= 2u^2), u = 2^-53.
// quad-double: component-wise two_sum / two_prod, the partial sums collected
// order by order (terms of order u^4 and below dropped), then a branch-free
// renormalisation made of exact two_sum "VecSum" passes.  The error of an
// add or multiply is O(2^-211) relative to the magnitude of the operands.
//
// Every routine is branch-free (the paper found the branching of its
// multiword library to hurt on the GPU).  Floating-point contraction must be
// off for this file: the transforms depend on each rounding being the one
// written, so every intended fused multiply-add is an explicit fma().
#pragma once

#include <hip/hip_runtime.h>
#include <cmath>

#pragma clang fp contract(off)

#define MPA __host__ __device__ __forceinline__

namespace lwk {

struct dd { double x0, x1; };
struct qd { double x0, x1, x2, x3; };

template <class T> struct words_of;
template <> struct words_of<double> { static constexpr int value = 1; };
template <> struct words_of<dd> { static constexpr int value = 2; };
template <> struct words_of<qd> { static constexpr int value = 4; };

// ------------------------------------------------------------------ EFTs
MPA void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double t = s - a;
    e = (a - (s - t)) + (b - t);
}
MPA void fast_two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    e = b - (s - a);
}
MPA void two_prod(double a, double b, double &p, double &e) {
    p = a * b;
    e = fma(a, b, -p);
}

// ------------------------------------------------------------------ double
MPA double mp_add(double a, double b) { return a + b; }
MPA double mp_sub(double a, double b) { return a - b; }
MPA double mp_mul(double a, double b) { return a * b; }
MPA double mp_mul_d(double a, double b) { return a * b; }
MPA double mp_madd(double a, double b, double c) { return fma(a, b, c); }   // a*b + c
MPA double mp_msub(double a, double b, double c) { return fma(-a, b, c); }  // c - a*b
MPA double mp_neg(double a) { return -a; }
MPA double mp_pow2(double a, double p2) { return a * p2; }                   // p2 a power of two
MPA double mp_lead(double a) { return a; }
template <class T> MPA T mp_from(double a);
template <> MPA double mp_from<double>(double a) { return a; }
MPA double mp_word(double a, int) { return a; }
MPA void mp_set_word(double &a, int, double v) { a = v; }

// ------------------------------------------------------------------ double-double
MPA dd mp_add(dd x, dd y) {
    double sh, sl, th, tl, vh, vl;
    two_sum(x.x0, y.x0, sh, sl);
    two_sum(x.x1, y.x1, th, tl);
    double c = sl + th;
    fast_two_sum(sh, c, vh, vl);
    double w = tl + vl;
    dd z;
    fast_two_sum(vh, w, z.x0, z.x1);
    return z;
}
MPA dd mp_neg(dd a) { return {-a.x0, -a.x1}; }
MPA dd mp_sub(dd x, dd y) { return mp_add(x, mp_neg(y)); }
MPA dd mp_mul(dd x, dd y) {
    double ch, cl1;
    two_prod(x.x0, y.x0, ch, cl1);
    double tl0 = x.x1 * y.x1;
    double tl1 = fma(x.x0, y.x1, tl0);
    double cl2 = fma(x.x1, y.x0, tl1);
    double cl3 = cl1 + cl2;
    dd z;
    fast_two_sum(ch, cl3, z.x0, z.x1);
    return z;
}
MPA dd mp_mul_d(dd x, double y) {
    double ch, cl1;
    two_prod(x.x0, y, ch, cl1);
    double cl3 = fma(x.x1, y, cl1);
    dd z;
    fast_two_sum(ch, cl3, z.x0, z.x1);
    return z;
}
MPA dd mp_madd(dd a, dd b, dd c) { return mp_add(mp_mul(a, b), c); }
MPA dd mp_msub(dd a, dd b, dd c) { return mp_sub(c, mp_mul(a, b)); }
MPA dd mp_pow2(dd a, double p2) { return {a.x0 * p2, a.x1 * p2}; }
MPA double mp_lead(dd a) { return a.x0; }
template <> MPA dd mp_from<dd>(double a) { return {a, 0.0}; }
MPA double mp_word(const dd &a, int w) { return w == 0 ? a.x0 : a.x1; }
MPA void mp_set_word(dd &a, int w, double v) { if (w == 0) a.x0 = v; else a.x1 = v; }

// ------------------------------------------------------------------ quad-double
// Branch-free renormalisation of x0 + x1 + x2 + x3 + x4 (roughly decreasing
// in magnitude, possibly overlapping) into four words.  Each VecSum pass
// (two_sum from the smallest term up) is exact and moves the leading part of
// what remains into the top word; four passes give the four output words,
// and only the last, plain addition rounds.
MPA qd qd_renorm(double x0, double x1, double x2, double x3, double x4) {
    double t, y1, y2, y3, y4, z0, z1, z2, w2, w3, w4, v3, v4;
    two_sum(x3, x4, t, y4);
    two_sum(x2, t, t, y3);
    two_sum(x1, t, t, y2);
    two_sum(x0, t, z0, y1);
    two_sum(y3, y4, t, w4);
    two_sum(y2, t, t, w3);
    two_sum(y1, t, z1, w2);
    two_sum(w3, w4, t, v4);
    two_sum(w2, t, z2, v3);
    return {z0, z1, z2, v3 + v4};
}

MPA qd mp_add(qd a, qd b) {
    double s0, s1, s2, s3, e0, e1, e2, e3, f1, f2, g;
    two_sum(a.x0, b.x0, s0, e0);
    two_sum(a.x1, b.x1, s1, e1);
    two_sum(a.x2, b.x2, s2, e2);
    two_sum(a.x3, b.x3, s3, e3);
    two_sum(s1, e0, s1, e0);        // order 1; e0 carries to order 2
    two_sum(s2, e1, s2, f1);        // order 2; f1, f2 carry to order 3
    two_sum(s2, e0, s2, f2);
    two_sum(s3, e2, s3, g);         // order 3; g, e3 are order 4
    s3 = s3 + (f1 + f2);
    return qd_renorm(s0, s1, s2, s3, e3 + g);
}
MPA qd mp_neg(qd a) { return {-a.x0, -a.x1, -a.x2, -a.x3}; }
MPA qd mp_sub(qd a, qd b) { return mp_add(a, mp_neg(b)); }

MPA qd mp_mul(qd a, qd b) {
    double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
    two_prod(a.x0, b.x0, p00, q00);                       // order 0 (+ order 1 error)
    two_prod(a.x0, b.x1, p01, q01);                       // order 1
    two_prod(a.x1, b.x0, p10, q10);
    two_prod(a.x0, b.x2, p02, q02);                       // order 2
    two_prod(a.x1, b.x1, p11, q11);
    two_prod(a.x2, b.x0, p20, q20);
    double s1, r1, r2, t;
    two_sum(p01, p10, t, r1);                             // order 1 collected
    two_sum(q00, t, s1, r2);
    double s2, ea, eb, ec, ed, ee, ef;                    // order 2 collected
    two_sum(q01, q10, t, ea);
    two_sum(t, p02, t, eb);
    two_sum(t, p11, t, ec);
    two_sum(t, p20, t, ed);
    two_sum(t, r1, t, ee);
    two_sum(t, r2, s2, ef);
    double o3 = fma(a.x0, b.x3, a.x1 * b.x2);             // order 3, rounded
    o3 = fma(a.x2, b.x1, o3);
    o3 = fma(a.x3, b.x0, o3);
    double s3 = ((q02 + q11) + q20) + o3 + (((ea + eb) + (ec + ed)) + (ee + ef));
    return qd_renorm(p00, s1, s2, s3, 0.0);
}

MPA qd mp_mul_d(qd a, double d) {
    double p0, q0, p1, q1, p2, q2, s1, r1, s2, r2, r3;
    two_prod(a.x0, d, p0, q0);
    two_prod(a.x1, d, p1, q1);
    two_prod(a.x2, d, p2, q2);
    two_sum(q0, p1, s1, r1);
    two_sum(q1, p2, s2, r2);
    two_sum(s2, r1, s2, r3);
    double s3 = fma(a.x3, d, q2) + (r2 + r3);
    return qd_renorm(p0, s1, s2, s3, 0.0);
}
MPA qd mp_madd(qd a, qd b, qd c) { return mp_add(mp_mul(a, b), c); }
MPA qd mp_msub(qd a, qd b, qd c) { return mp_sub(c, mp_mul(a, b)); }
MPA qd mp_pow2(qd a, double p2) { return {a.x0 * p2, a.x1 * p2, a.x2 * p2, a.x3 * p2}; }
MPA double mp_lead(qd a) { return a.x0; }
template <> MPA qd mp_from<qd>(double a) { return {a, 0.0, 0.0, 0.0}; }
MPA double mp_word(const qd &a, int w) {
    return w == 0 ? a.x0 : w == 1 ? a.x1 : w == 2 ? a.x2 : a.x3;
}
MPA void mp_set_word(qd &a, int w, double v) {
    if (w == 0) a.x0 = v; else if (w == 1) a.x1 = v; else if (w == 2) a.x2 = v; else a.x3 = v;
}

// ------------------------------------------------------------------ complex
template <class T> struct cx { T re, im; };

template <class T> MPA cx<T> c_add(cx<T> a, cx<T> b) { return {mp_add(a.re, b.re), mp_add(a.im, b.im)}; }
template <class T> MPA cx<T> c_sub(cx<T> a, cx<T> b) { return {mp_sub(a.re, b.re), mp_sub(a.im, b.im)}; }
template <class T> MPA cx<T> c_pow2(cx<T> a, double p2) { return {mp_pow2(a.re, p2), mp_pow2(a.im, p2)}; }
// (zr + i zi) * a
template <class T> MPA cx<T> c_mul(T zr, T zi, cx<T> a) {
    return {mp_msub(zi, a.im, mp_mul(zr, a.re)), mp_madd(zi, a.re, mp_mul(zr, a.im))};
}
// acc + (zr + i zi) * a
template <class T> MPA cx<T> c_madd(T zr, T zi, cx<T> a, cx<T> acc) {
    return {mp_msub(zi, a.im, mp_madd(zr, a.re, acc.re)), mp_madd(zi, a.re, mp_madd(zr, a.im, acc.im))};
}
// acc - (zr + i zi) * a
template <class T> MPA cx<T> c_msub(T zr, T zi, cx<T> a, cx<T> acc) {
    return {mp_madd(zi, a.im, mp_msub(zr, a.re, acc.re)), mp_msub(zi, a.re, mp_msub(zr, a.im, acc.im))};
}
// acc + x * a (x real)
template <class T> MPA cx<T> c_rmadd(T x, cx<T> a, cx<T> acc) { return {mp_madd(x, a.re, acc.re), mp_madd(x, a.im, acc.im)}; }
template <class T> MPA cx<T> c_rmsub(T x, cx<T> a, cx<T> acc) { return {mp_msub(x, a.re, acc.re), mp_msub(x, a.im, acc.im)}; }

}  // namespace lwk
