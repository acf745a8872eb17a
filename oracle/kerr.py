"""Kerr background factors of the 2+1D Teukolsky system, >= 400 bits (test infrastructure).

Everything here follows Sec. "Teukolsky Code" of the paper:

* tortoise coordinate  dr*/dr = (r^2+a^2)/Delta, Delta = r^2 - 2Mr + a^2
  (the paper fixes only the differential; the integration constant used here
  is the standard one, see ``tortoise``);
* azimuthal coordinate dphi~ = dphi + a/Delta dr and the ansatz
  Psi = exp(i m phi~) r^3 Phi(t, r*, theta)  (Eq. (psiphi));
* Pi = d_t Phi + b d_r* Phi,  b = (r^2+a^2)/Sigma,
  Sigma^2 = (r^2+a^2)^2 - a^2 Delta sin^2 theta.

The paper defers the explicit matrices M, L, A of its first-order form (Eq.
(evln)) to the literature.  Written for the complex pair (Phi, Pi) the system
is

    d_t Phi + b d_r* Phi = Pi
    d_t Pi  - b d_r* Pi  = -K d_r* Phi + W Lth Phi + C0 Phi - Ct Pi

so that, with u = (Phi_R, Phi_I, Pi_R, Pi_I) and D = diag(b, b, -b, -b)
(Eq. (d_matrix)), the source S of Eq. (new_teu2) is S_Phi = Pi and S_Pi as
above.  Lth is the angular operator of Eq. (1) after the ansatz:

    Lth Phi = Phi_thth + cot(theta) Phi_th - [(m + s cos theta)^2 / sin^2 theta - s] Phi.

The coefficient formulas below were obtained by substituting the ansatz into
Eq. (1) and dividing by the coefficient of the second time derivative;
tests/test_oracle_kerr.py checks them against Eq. (1) itself by numerical
differentiation at high precision (a pin that does not reuse them).
"""
import mpmath as mp

WORK_BITS = 450          # working precision of every function here


def _mpf(x):
    return x if isinstance(x, mp.mpf) else mp.mpf(x)


def horizons(M, a):
    """(r_plus, r_minus) = M +- sqrt(M^2 - a^2); requires |a| < M (or M = a = 0)."""
    M, a = _mpf(M), _mpf(a)
    d = mp.sqrt(M * M - a * a)
    return M + d, M - d


def tortoise(r, M, a):
    """r*(r) for r > r_plus.

    Integrating dr*/dr = (r^2+a^2)/Delta by partial fractions gives

      r* = r + 2M r+/(r+ - r-) ln((r - r+)/2M) - 2M r-/(r+ - r-) ln((r - r-)/2M)

    (a = 0: r + 2M ln(r/2M - 1); M = 0, flat space: r* = r).
    """
    r, M, a = _mpf(r), _mpf(M), _mpf(a)
    if M == 0:
        if a != 0:
            raise ValueError("flat space needs a = 0")
        return r
    rp, rm = horizons(M, a)
    out = r + 2 * M * rp / (rp - rm) * mp.log((r - rp) / (2 * M))
    if rm != 0:
        out -= 2 * M * rm / (rp - rm) * mp.log((r - rm) / (2 * M))
    return out


def r_of_tortoise(rs, M, a):
    """Invert ``tortoise``: the unique r > r_plus with r*(r) = rs.

    r*(r) is strictly increasing on (r_plus, inf) (its derivative is
    (r^2+a^2)/Delta > 0), running from -inf to +inf, so the root is
    bracketed and found by bisection on x = r - r_plus (in log scale) and
    then polished by Newton steps until the correction is below the working
    precision.
    """
    rs, M, a = _mpf(rs), _mpf(M), _mpf(a)
    if M == 0:
        return rs
    rp, rm = horizons(M, a)

    def f(x):                      # r*(r_plus + x) - rs
        return tortoise(rp + x, M, a) - rs

    lo, hi = mp.mpf(-1), mp.mpf(1)        # bracket in ln x
    while f(mp.exp(lo)) > 0:
        lo *= 2
    while f(mp.exp(hi)) < 0:
        hi *= 2
    for _ in range(60):                   # bisection to ~double accuracy
        mid = (lo + hi) / 2
        if f(mp.exp(mid)) > 0:
            hi = mid
        else:
            lo = mid
    r = rp + mp.exp((lo + hi) / 2)
    eps = mp.ldexp(1, -mp.mp.prec + 8)
    for _ in range(40):                   # Newton: dr = -(r*(r) - rs) Delta / varpi
        delta = (r - rp) * (r - rm)
        step = (tortoise(r, M, a) - rs) * delta / (r * r + a * a)
        r -= step
        if abs(step) <= eps * r:
            break
    else:
        raise ArithmeticError("tortoise inversion did not converge")
    return r


def background(r, cos_t, sin2_t, s, m, M, a):
    """Coefficients of the first-order system at Boyer-Lindquist radius r.

    Returns a dict of mp numbers:
      b   = varpi / Sigma                          (real)
      W   = Delta / Sigma^2                        (real)
      Ct  = [4 i M a m r + 2 s (r Delta - M (r^2 - a^2)) + 2 i s a Delta cos] / Sigma^2
      C0  = W [6 Delta / r^2 + 3 ((s+1) Delta' + 2 i a m) / r] + 4 i a m s (r - M) / Sigma^2
      Cs  = W (6 varpi / r + 2 r) + (varpi / Sigma^2)(s Delta' + 2 i a m)
      bdb = b d_r* b = a^2 Delta sin^2 (varpi Delta' - 4 r Delta) / (2 Sigma^4)
      K   = bdb - b Ct - Cs
    where varpi = r^2 + a^2, Delta' = 2 (r - M).  After eliminating Pi the
    system reads Phi_tt - b^2 Phi_r*r* + Ct Phi_t - Cs Phi_r* - W Lth Phi - C0 Phi = 0,
    which is Eq. (1) divided by -(Sigma^2/Delta) r^3 exp(i m phi~).
    ``cos_t`` and ``sin2_t`` are cos(theta) and sin(theta)^2.
    """
    r, M, a = _mpf(r), _mpf(M), _mpf(a)
    s, m = int(s), int(m)
    I = mp.mpc(0, 1)
    varpi = r * r + a * a
    delta = r * r - 2 * M * r + a * a
    ddelta = 2 * (r - M)
    sig2 = varpi * varpi - a * a * delta * sin2_t
    sig = mp.sqrt(sig2)
    b = varpi / sig
    W = delta / sig2
    Ct = (4 * I * M * a * m * r + 2 * s * (r * delta - M * (r * r - a * a))
          + 2 * I * s * a * delta * cos_t) / sig2
    C0 = W * (6 * delta / (r * r) + 3 * ((s + 1) * ddelta + 2 * I * a * m) / r) \
        + 4 * I * a * m * s * (r - M) / sig2
    Cs = W * (6 * varpi / r + 2 * r) + varpi / sig2 * (s * ddelta + 2 * I * a * m)
    bdb = a * a * delta * sin2_t * (varpi * ddelta - 4 * r * delta) / (2 * sig2 * sig2)
    K = bdb - b * Ct - Cs
    return {"b": b, "W": W, "Ct": mp.mpc(Ct), "C0": mp.mpc(C0), "Cs": mp.mpc(Cs),
            "bdb": bdb, "K": mp.mpc(K), "Sigma2": sig2, "Delta": delta, "varpi": varpi}


def angular_potential(cos_t, sin2_t, s, m):
    """V(theta) = s - (m + s cos theta)^2 / sin^2 theta, the undifferentiated part of Lth."""
    return s - (m + s * cos_t) ** 2 / sin2_t
