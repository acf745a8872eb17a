// Division, square root, exp, log, sin and cos in double / double-double /
// quad-double, for the once-per-grid coefficient pass (tortoise inversion,
// Kerr factors, angular grid).  None of these is on the per-step path, so
// they favour simple, robust formulations over speed:
//
//   div    Newton iteration for the reciprocal from the double reciprocal,
//          then one correction of the quotient
//   sqrt   Newton iteration y += (x - y^2) / (2 y0) from the double root
//   exp    reduction x = k ln2 + r (|r| <= ln2/2), Taylor series of e^r in
//          Horner form, scaling by 2^k; no squaring steps, so no error growth
//   log    Newton iteration on exp: y += x e^-y - 1 from the double log
//   sincos Taylor series on |x| <= pi/2 (the angular grid needs no more)
//
// Each Newton step at least doubles the number of correct bits, so
// words + 1 steps reach full precision from a 53-bit start.
#pragma once

#include "mparith.hpp"

#pragma clang fp contract(off)

namespace lwk {

// pi and ln 2 as non-overlapping four-word expansions
template <class T> MPA T mp_const_pi();
template <class T> MPA T mp_const_ln2();
template <> MPA double mp_const_pi<double>() { return 0x1.921fb54442d18p+1; }
template <> MPA dd mp_const_pi<dd>() { return {0x1.921fb54442d18p+1, 0x1.1a62633145c07p-53}; }
template <> MPA qd mp_const_pi<qd>() {
    return {0x1.921fb54442d18p+1, 0x1.1a62633145c07p-53, -0x1.f1976b7ed8fbcp-109, 0x1.4cf98e804177dp-163};
}
template <> MPA double mp_const_ln2<double>() { return 0x1.62e42fefa39efp-1; }
template <> MPA dd mp_const_ln2<dd>() { return {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56}; }
template <> MPA qd mp_const_ln2<qd>() {
    return {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56, 0x1.7b57a079a1934p-111, -0x1.ace93a4ebe5d1p-165};
}

template <class T> MPA T mp_one() { return mp_from<T>(1.0); }

template <class T> MPA T mp_recip(T b) {
    T y = mp_from<T>(1.0 / mp_lead(b));
    for (int it = 0; it < words_of<T>::value; ++it)           // y += y (1 - b y)
        y = mp_madd(y, mp_msub(b, y, mp_one<T>()), y);
    return y;
}

template <class T> MPA T mp_div(T a, T b) {
    T y = mp_recip(b);
    T q = mp_mul(a, y);
    return mp_madd(y, mp_msub(b, q, a), q);                    // q += y (a - b q)
}

template <class T> MPA T mp_div_d(T a, double d) { return mp_div(a, mp_from<T>(d)); }

template <class T> MPA T mp_sqrt(T x) {
    double x0 = mp_lead(x);
    if (!(x0 > 0.0)) return mp_from<T>(0.0);
    double r0 = sqrt(x0);
    T y = mp_from<T>(r0);
    double h = 0.5 / r0;
    for (int it = 0; it < words_of<T>::value + 1; ++it)        // y += (x - y^2) / (2 y0)
        y = mp_add(y, mp_mul_d(mp_msub(y, y, x), h));
    return y;
}

// number of Taylor terms that make the truncation error negligible
template <class T> struct series_terms;
template <> struct series_terms<double> { static constexpr int exp = 18, trig = 13; };
template <> struct series_terms<dd> { static constexpr int exp = 30, trig = 22; };
template <> struct series_terms<qd> { static constexpr int exp = 52, trig = 36; };

template <class T> MPA T mp_exp(T x) {
    const double kf = rint(mp_lead(x) / 0x1.62e42fefa39efp-1);
    T r = mp_msub(mp_const_ln2<T>(), mp_from<T>(kf), x);      // x - k ln2
    // Horner: 1 + r (1 + r/2 (1 + r/3 (...)))
    T acc = mp_one<T>();
    for (int n = series_terms<T>::exp; n >= 1; --n)
        acc = mp_add(mp_one<T>(), mp_div_d(mp_mul(r, acc), (double)n));
    return mp_pow2(acc, ldexp(1.0, (int)kf));
}

template <class T> MPA T mp_log(T x) {
    T y = mp_from<T>(log(mp_lead(x)));
    for (int it = 0; it < words_of<T>::value; ++it)            // y += x e^-y - 1
        y = mp_add(y, mp_sub(mp_mul(x, mp_exp(mp_neg(y))), mp_one<T>()));
    return y;
}

// sin and cos of x, |x| <= pi/2
template <class T> MPA void mp_sincos(T x, T &s, T &c) {
    T x2 = mp_mul(x, x);
    const int N = series_terms<T>::trig;
    T ss = mp_one<T>(), cc = mp_one<T>();
    for (int n = N; n >= 1; --n) {
        // sin x = x (1 - x^2/(2*3) (1 - x^2/(4*5) (...)));  cos x = 1 - x^2/(1*2) (1 - x^2/(3*4) (...))
        ss = mp_sub(mp_one<T>(), mp_div_d(mp_mul(x2, ss), (double)(2 * n) * (double)(2 * n + 1)));
        cc = mp_sub(mp_one<T>(), mp_div_d(mp_mul(x2, cc), (double)(2 * n - 1) * (double)(2 * n)));
    }
    s = mp_mul(x, ss);
    c = cc;
}

}  // namespace lwk
