// Fused multiword dot products: acc = sum_k a_k * b_k + sum_l v_l, rounded to T
// once at the end.  The stencil and every output of a Lax-Wendroff stage are
// such sums, so collecting their partial products order by order and
// normalising once replaces a renormalising multiply and add per term.
//
// double: a chain of FMAs.
// double-double: the products' leading parts are summed exactly (two_prod
//   and two_sum, errors pushed to the next order); all order-u terms (product
//   errors, cross products, low words, two_sum errors) go into one double.
//   Absolute error O(u^2) sum_k |a_k b_k| + O(u^2) sum_l |v_l|, the same order
//   as a sequence of double-double operations (Ogita-Rump-Oishi compensated
//   dot product, extended to double-double inputs).
// quad-double: four running sums s0..s3, one per order u^0..u^3; the terms of
//   orders 0, 1 and 2 are added with two_sum and their errors passed one order
//   down, the order-3 terms with plain additions; the product terms of order
//   4 and below are dropped.  Absolute error O(u^4) (sum |a_k b_k| + sum |v_l|).
// In quad-double a product's own lower-order terms are first combined among
// themselves (exactly where the order requires it), off the running sums'
// dependency chains: each running sum then sees two to four additions per
// product instead of up to ten, so consecutive products overlap in the
// pipeline (measured: 4 % faster on the 2048 x 64 grid; the same treatment of
// the double-double sum gained nothing).
//
// Operands are non-overlapping expansions; results are renormalised.
#pragma once

#include "mparith.hpp"

#pragma clang fp contract(off)

namespace lwk {

template <class T> struct Acc;

template <> struct Acc<double> {
    // starts at -0: -0 + v == v and fma(a, b, -0) == a*b for every v, a*b
    // (signed zeros included), so the compiler drops the first addition
    double s = -0.0;
    MPA void prod(double a, double b) { s = fma(a, b, s); }
    MPA void value(double v) { s += v; }
    MPA double result() const { return s; }
};

template <> struct Acc<dd> {
    double s = 0.0, c = 0.0;
    MPA void prod(const dd &a, const dd &b) {
        double p, e, t;
        two_prod(a.x0, b.x0, p, e);
        two_sum(s, p, s, t);
        c = fma(a.x0, b.x1, fma(a.x1, b.x0, c + (t + e)));
    }
    MPA void value(const dd &v) {
        double t;
        two_sum(s, v.x0, s, t);
        c += t + v.x1;
    }
    MPA dd result() const {
        dd z;
        two_sum(s, c, z.x0, z.x1);
        return z;
    }
};

template <> struct Acc<qd> {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    // add x at order 1 / 2 (exactly, error one order down) or order 3 (rounded)
    MPA void o1(double x) { double t; two_sum(s1, x, s1, t); o2(t); }
    MPA void o2(double x) { double t; two_sum(s2, x, s2, t); s3 += t; }
    MPA void prod(const qd &a, const qd &b) {
        double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20, t;
        two_prod(a.x0, b.x0, p00, q00);
        two_prod(a.x0, b.x1, p01, q01);
        two_prod(a.x1, b.x0, p10, q10);
        two_prod(a.x0, b.x2, p02, q02);
        two_prod(a.x1, b.x1, p11, q11);
        two_prod(a.x2, b.x0, p20, q20);
        // order 1 of the product: p01 + p10 + q00 = u1 + (e1 + e2 at order 2)
        double u1, e1, e2;
        two_sum(p01, p10, u1, e1);
        two_sum(u1, q00, u1, e2);
        // order 2: p02 + p11 + p20 + q01 + q10 + e1 + e2 = u2 + (f1..f6 at order 3)
        double u2, v2, v3, f1, f2, f3, f4, f5, f6;
        two_sum(p02, p11, u2, f1);
        two_sum(p20, q01, v2, f2);
        two_sum(q10, e1, v3, f3);
        two_sum(u2, v2, u2, f4);
        two_sum(v3, e2, v3, f5);
        two_sum(u2, v3, u2, f6);
        // order 3, rounded
        double o3 = fma(a.x0, b.x3, a.x1 * b.x2);
        o3 = fma(a.x2, b.x1, o3);
        o3 = fma(a.x3, b.x0, o3);
        const double u3 = (((q02 + q11) + q20) + o3) + (((f1 + f2) + (f3 + f4)) + (f5 + f6));
        two_sum(s0, p00, s0, t);
        o1(t);
        o1(u1);
        o2(u2);
        s3 += u3;
    }
    MPA void value(const qd &v) {
        double t;
        two_sum(s0, v.x0, s0, t);
        o1(t);
        o1(v.x1);
        o2(v.x2);
        s3 += v.x3;
    }
    MPA qd result() const { return qd_renorm(s0, s1, s2, s3, 0.0); }
};

// sloppy two-operand sums for neighbour averages and differences: the
// absolute error is O(u^words) (|a| + |b|), which is what the scheme needs
// (its outputs are measured against the largest field value)
MPA double mp_add_fast(double a, double b) { return a + b; }
MPA dd mp_add_fast(const dd &a, const dd &b) {
    double s, e;
    two_sum(a.x0, b.x0, s, e);
    e += a.x1 + b.x1;
    dd z;
    fast_two_sum(s, e, z.x0, z.x1);
    return z;
}
MPA qd mp_add_fast(const qd &a, const qd &b) { return mp_add(a, b); }

}  // namespace lwk
