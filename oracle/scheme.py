"""The two-step Lax-Wendroff update, written out point by point (test infrastructure).

Plain Python loops over a generic number type: with ``fractions.Fraction``
tables and fields it is exact (the brute-force pin of the fixed-point
engine); with mpmath numbers it runs at their precision.  Only for tiny grids.

Notation follows Sec. "Teukolsky Code": u = (Phi_R, Phi_I, Pi_R, Pi_I) is
kept as two complex pairs (Phi, Pi); D = diag(b, b, -b, -b) acts as +b on
Phi and -b on Pi; the source is S_Phi = Pi,
S_Pi = -K d_r* Phi + W Lth Phi + C0 Phi - Ct Pi (see oracle.kerr).

  (lw1)  u^{n+1/2}_{i+1/2} = 1/2 (u^n_{i+1} + u^n_i)
                             - dt/2 [ D_{i+1/2} (u^n_{i+1} - u^n_i)/dr* - S^n_{i+1/2} ]
  (lw2)  u^{n+1}_i = u^n_i - dt [ D_i (u^{n+1/2}_{i+1/2} - u^{n+1/2}_{i-1/2})/dr* - S^{n+1/2}_i ]

Reading of the staggering (the paper labels S by the point only): the source
at a point where the stage has no grid value uses the average of the two
neighbouring values and their difference over dr* for the radial
derivative; coefficients are evaluated at that point.  Radial boundary:
u = 0 at i = 0 and i = n_r-1 after every step.  Angular boundary: ghost rows
beyond each pole are mirror images times (-1)^|m| (even |m|: zero slope,
odd |m|: zero value at the pole).
"""


def _add(a, b):
    return (a[0] + b[0], a[1] + b[1])


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def _rmul(x, a):                 # real * complex
    return (x * a[0], x * a[1])


def _cmul(z, a):                 # complex * complex
    return (z[0] * a[0] - z[1] * a[1], z[0] * a[1] + z[1] * a[0])


def as_pairs(tables):
    """Copy of ``tables`` with every complex entry given as a (re, im) pair."""
    def pair(z):
        return (z.real, z.imag) if hasattr(z, "imag") and not isinstance(z, tuple) else z
    out = dict(tables)
    for key in ("half", "full"):
        out[key] = [[(pt[0], pt[1]) + tuple(pair(v) for v in pt[2:]) for pt in row]
                    for row in tables[key]]
    return out


def theta_operator(col, j, T):
    """Lth applied to the column ``col`` (complex pairs over theta rows) at row j.

    Lth Phi = Phi_thth + cot(theta) Phi_th + V(theta) Phi with centred
    differences of reach R; ghost rows by reflection with sign (-1)^|m|.
    """
    n = len(col)
    R = T["reach"]
    P = T["parity"]

    def g(q):
        if q < 0:
            v = col[-1 - q]
        elif q >= n:
            v = col[2 * n - 1 - q]
        else:
            return col[q]
        return v if P == 1 else (-v[0], -v[1])

    zero = col[j][0] * 0
    d2 = (zero, zero)
    d1 = (zero, zero)
    for k in range(-R, R + 1):
        v = g(j + k)
        d2 = _add(d2, _rmul(T["d2"][k + R], v))
        d1 = _add(d1, _rmul(T["d1"][k + R], v))
    return _add(_add(d2, _rmul(T["cot"][j], d1)), _rmul(T["V"][j], col[j]))


def lw_step(phi, pi, T, half):
    """One full step.  phi, pi: lists [j][i] of complex pairs; returns new (phi, pi).

    ``half`` is 1/2 in the number type in use.
    """
    nth = len(phi)
    nr = len(phi[0])
    inv_h, dt = T["inv_h"], T["dt"]
    hdt = half * dt
    # ---- (lw1): half step at r*_{i+1/2}, i = 0..nr-2
    phih = [[None] * (nr - 1) for _ in range(nth)]
    pih = [[None] * (nr - 1) for _ in range(nth)]
    for i in range(nr - 1):
        phibar = [_rmul(half, _add(phi[j][i + 1], phi[j][i])) for j in range(nth)]
        pibar = [_rmul(half, _add(pi[j][i + 1], pi[j][i])) for j in range(nth)]
        for j in range(nth):
            b, W, K, Ct, C0 = T["half"][j][i]
            dphi = _rmul(inv_h, _sub(phi[j][i + 1], phi[j][i]))
            dpi = _rmul(inv_h, _sub(pi[j][i + 1], pi[j][i]))
            lth = theta_operator(phibar, j, T)
            s_phi = pibar[j]
            s_pi = _add(_sub(_add(_rmul(-1, _cmul(K, dphi)), _rmul(W, lth)), _cmul(Ct, pibar[j])),
                        _cmul(C0, phibar[j]))
            phih[j][i] = _sub(phibar[j], _rmul(hdt, _sub(_rmul(b, dphi), s_phi)))
            pih[j][i] = _sub(pibar[j], _rmul(hdt, _sub(_rmul(-b, dpi), s_pi)))
    # ---- (lw2): full step at interior r*_i, i = 1..nr-2
    zero = (phi[0][0][0] * 0, phi[0][0][0] * 0)
    nphi = [[zero] * nr for _ in range(nth)]
    npi = [[zero] * nr for _ in range(nth)]
    for i in range(1, nr - 1):
        phim = [_rmul(half, _add(phih[j][i], phih[j][i - 1])) for j in range(nth)]
        pim = [_rmul(half, _add(pih[j][i], pih[j][i - 1])) for j in range(nth)]
        for j in range(nth):
            b, W, K, Ct, C0 = T["full"][j][i]
            dphi = _rmul(inv_h, _sub(phih[j][i], phih[j][i - 1]))
            dpi = _rmul(inv_h, _sub(pih[j][i], pih[j][i - 1]))
            lth = theta_operator(phim, j, T)
            s_phi = pim[j]
            s_pi = _add(_sub(_add(_rmul(-1, _cmul(K, dphi)), _rmul(W, lth)), _cmul(Ct, pim[j])),
                        _cmul(C0, phim[j]))
            nphi[j][i] = _sub(phi[j][i], _rmul(dt, _sub(_rmul(b, dphi), s_phi)))
            npi[j][i] = _sub(pi[j][i], _rmul(dt, _sub(_rmul(-b, dpi), s_pi)))
    return nphi, npi


def evolve(phi, pi, T, nsteps, half):
    for _ in range(nsteps):
        phi, pi = lw_step(phi, pi, T, half)
    return phi, pi
