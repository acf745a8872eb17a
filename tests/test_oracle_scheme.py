"""Pins of the oracle's Lax-Wendroff scheme (Python form and C fixed-point engine).

* exact rationals: the fixed-point engine equals exact Fraction arithmetic to
  its rounding (pins the engine's arithmetic against the literal scheme);
* flat space (M = a = s = 0): closed-form outgoing multipoles, error -> 0 at
  second order under refinement (pins the discretisation end to end);
* the angular operator converges at the stated tenth order on smooth data
  with the pole behaviour the reflection assumes;
* linearity, reality at a = 0, conjugation-reflection symmetry m -> -m,
  theta -> pi - theta, and zero radial boundaries.
"""
from fractions import Fraction
import math
import random

import mpmath as mp
import numpy as np
import pytest

from oracle import engine, problem, scheme

FRAC = engine.FRAC


def _rand_state(nth, nr, seed):
    random.seed(seed)
    rnd = lambda: Fraction(random.randint(-2 ** 60, 2 ** 60), 2 ** 60)
    phi = [[(rnd(), rnd()) for _ in range(nr)] for _ in range(nth)]
    pi = [[(rnd(), rnd()) for _ in range(nr)] for _ in range(nth)]
    for f in (phi, pi):
        for row in f:
            row[0] = row[-1] = (Fraction(0), Fraction(0))
    return phi, pi


def _flat_ints(phi, pi):
    out = []
    for c in range(4):
        src = phi if c < 2 else pi
        out += [engine.mp_to_fixed(row[i][c % 2]) for row in src for i in range(len(row))]
    return out


@pytest.mark.parametrize("s,m,a,order", [(-2, 1, 0.7, 10), (-2, 2, 0.5, 10), (0, 0, 0.0, 2), (1, -3, 0.95, 10)])
def test_engine_matches_exact_rationals(s, m, a, order):
    p = problem.Problem(s=s, m=m, a_over_M=a, n_r=8, n_theta=6, rstar_min=-10, rstar_max=30,
                        angular_order=order)
    TF = problem.to_fractions(problem.build_tables(p), bits=100)
    phi, pi = _rand_state(p.n_theta, p.n_r, 3 + m)
    ephi, epi = scheme.evolve(phi, pi, TF, 3, Fraction(1, 2))
    out = engine.run_fixed(engine.tables_to_fixed(TF), p.n_r, p.n_theta, _flat_ints(phi, pi), 3)
    exact = _flat_ints(ephi, epi)           # exact values rounded to 2^-384
    mx = max(abs(v) for v in exact)
    err = max(abs(x - y) for x, y in zip(out, exact))
    assert err <= mx * 2 ** -375, math.log2(err / mx)


def test_engine_rejects_planted_scheme_change():
    """A dropped source term in the exact scheme must show as a large difference."""
    p = problem.Problem(s=-2, m=2, a_over_M=0.5, n_r=8, n_theta=6, rstar_min=-10, rstar_max=30)
    TF = problem.to_fractions(problem.build_tables(p), bits=100)
    phi, pi = _rand_state(p.n_theta, p.n_r, 7)
    bad = dict(TF)
    bad["half"] = [[(b, W, K, Ct, (Fraction(0), Fraction(0))) for (b, W, K, Ct, C0) in row] for row in TF["half"]]
    ephi, epi = scheme.evolve(phi, pi, bad, 2, Fraction(1, 2))
    out = engine.run_fixed(engine.tables_to_fixed(TF), p.n_r, p.n_theta, _flat_ints(phi, pi), 2)
    exact = _flat_ints(ephi, epi)
    mx = max(abs(v) for v in exact)
    assert max(abs(x - y) for x, y in zip(out, exact)) > mx * 1e-6


# ---------------------------------------------------------------- flat space
def _flat_solution(ell, t, r, th):
    """Outgoing multipole of the flat wave equation with s = m = 0:
    Psi = r^l (r^-1 d_r)^l [f(t - r)/r] P_l(cos th), Phi = Psi / r^3,
    Pi = Phi_t + Phi_r (b = 1).  f is a Gaussian centred at t - r = -8."""
    f = lambda u: mp.exp(-(u + 8) ** 2)

    def psi_rad(t, r):
        g = lambda rr: f(t - rr) / rr
        for _ in range(ell):
            g = (lambda gg: (lambda rr: mp.diff(gg, rr) / rr))(g)
        return r ** ell * g(r)

    Pl = mp.legendre(ell, mp.cos(th))
    phi = lambda tt, rr: psi_rad(tt, rr) / rr ** 3
    val = phi(t, r)
    pi = mp.diff(lambda tt: phi(tt, r), t) + mp.diff(lambda rr: phi(t, rr), r)
    return val * Pl, pi * Pl


def _flat_error(nr, nth, T, ells=(0, 1)):
    p = problem.Problem(s=0, m=0, a_over_M=0.0, n_r=nr, n_theta=nth, rstar_min=2.0, rstar_max=14.0,
                        mass=0.0)
    tab = problem.build_tables(p)
    dt, h, k = tab["dt"], tab["h"], tab["dtheta"]
    nsteps = int(mp.nint(T / dt))
    assert abs(nsteps * dt - T) < 1e-30
    with mp.workprec(200):
        cache = {}

        def sol(t, i, j):
            key = (t, i, j)
            if key not in cache:
                r, th = 2 + i * h, (j + mp.mpf(1) / 2) * k
                s = [_flat_solution(l, t, r, th) for l in ells]
                cache[key] = (sum(x[0] for x in s), sum(x[1] for x in s))
            return cache[key]
        # radial profiles are separable: evaluate on columns once per row class
        u0 = [0] * (4 * nth * nr)
        uT = [0] * (4 * nth * nr)
        for j in range(nth):
            for i in range(1, nr - 1):
                for (t, arr) in ((mp.mpf(0), u0), (mp.mpf(T), uT)):
                    ph, pi = sol(t, i, j)
                    arr[0 * nth * nr + j * nr + i] = engine.mp_to_fixed(ph)
                    arr[2 * nth * nr + j * nr + i] = engine.mp_to_fixed(pi)
    out = engine.run_fixed(engine.tables_to_fixed(tab), nr, nth, u0, nsteps)
    n = nth * nr
    err = max(abs(out[q] - uT[q]) for q in range(n))          # Phi_R
    mx = max(abs(uT[q]) for q in range(n))
    return err / mx


@pytest.mark.slow
def test_flat_space_closed_form_second_order():
    e = [_flat_error(nr, nth, 2) for nr, nth in ((61, 8), (121, 16), (241, 32))]
    o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
    assert e[2] < 1e-2
    assert 1.8 < o1 < 2.3 and 1.85 < o2 < 2.2, (e, o1, o2)


# ---------------------------------------------------------------- angular operator
@pytest.mark.parametrize("s,m", [(-2, 2), (-2, 1), (0, 0), (2, -3)])
def test_theta_operator_tenth_order(s, m):
    """Lth on smooth data with the pole parity (-1)^m, against Lth evaluated
    by numerical differentiation of the exact function.  Tenth order in the
    interior; in the rows next to a pole cot(theta) ~ 2/dtheta multiplies the
    first-derivative error, so the max-norm order there is nine."""
    with mp.workprec(300):
        def fun(th):
            return mp.sin(th) ** abs(m) * mp.exp(mp.mpf("0.3") * mp.cos(th))

        def exact_L(th):
            return (mp.diff(fun, th, 2) + mp.cos(th) / mp.sin(th) * mp.diff(fun, th)
                    + (s - (m + s * mp.cos(th)) ** 2 / mp.sin(th) ** 2) * fun(th))
        errs = []
        for nth in (32, 64):
            p = problem.Problem(s=s, m=m, a_over_M=0.0, n_r=3, n_theta=nth, rstar_min=-1, rstar_max=1)
            tab = problem.build_tables(p)
            k = tab["dtheta"]
            col = [(fun((j + mp.mpf(1) / 2) * k), mp.mpf(0)) for j in range(nth)]
            errs.append(max(abs(scheme.theta_operator(col, j, tab)[0] - exact_L((j + mp.mpf(1) / 2) * k))
                            for j in range(nth)))
        order = math.log2(float(errs[0] / errs[1]))
        assert order > 8.5, (errs, order)


# ---------------------------------------------------------------- properties
def _small_problem(**kw):
    base = dict(s=-2, m=2, a_over_M=0.6, n_r=24, n_theta=12, rstar_min=-20.0, rstar_max=40.0)
    base.update(kw)
    return problem.Problem(**base)


def _rand_fields(p, seed, real=False):
    rng = np.random.default_rng(seed)
    f = [rng.standard_normal((p.n_theta, p.n_r)) for _ in range(4)]
    if real:
        f[1][:] = 0
        f[3][:] = 0
    for a in f:
        a[:, 0] = a[:, -1] = 0
    return f


def test_linearity():
    p = _small_problem()
    tab = problem.build_tables(p)
    FT = engine.tables_to_fixed(tab)
    u = engine.fields_to_fixed(_rand_fields(p, 1))
    v = engine.fields_to_fixed(_rand_fields(p, 2))
    w = [3 * x - 5 * y for x, y in zip(u, v)]
    ru, rv, rw = (engine.run_fixed(FT, p.n_r, p.n_theta, z, 6) for z in (u, v, w))
    mx = max(abs(x) for x in rw)
    assert max(abs(3 * x - 5 * y - z) for x, y, z in zip(ru, rv, rw)) < mx * 2 ** -370


def test_schwarzschild_real_data_stays_real():
    p = _small_problem(a_over_M=0.0)
    out = engine.run_problem(p, _rand_fields(p, 3, real=True), 6)
    n = p.n_r * p.n_theta
    assert all(v == 0 for v in out[n:2 * n]) and all(v == 0 for v in out[3 * n:])
    assert any(v != 0 for v in out[:n])


def test_conjugation_reflection_symmetry():
    """(m, u(theta)) and (-m, conj u(pi - theta)) evolve into each other."""
    p = _small_problem(m=1, a_over_M=0.8)
    q = _small_problem(m=-1, a_over_M=0.8)
    f = _rand_fields(p, 4)
    g = [f[0][::-1].copy(), -f[1][::-1], f[2][::-1].copy(), -f[3][::-1]]
    op = engine.run_problem(p, f, 5)
    oq = engine.run_problem(q, g, 5)
    n, nr, nth = p.n_r * p.n_theta, p.n_r, p.n_theta
    mx = max(abs(v) for v in op)
    worst = 0
    for c, sign in enumerate((1, -1, 1, -1)):
        for j in range(nth):
            for i in range(nr):
                a = op[c * n + j * nr + i]
                b = oq[c * n + (nth - 1 - j) * nr + i]
                worst = max(worst, abs(a - sign * b))
    assert worst < mx * 2 ** -370


def test_radial_boundaries_stay_zero():
    p = _small_problem()
    out = engine.run_problem(p, _rand_fields(p, 5), 4)
    n, nr = p.n_r * p.n_theta, p.n_r
    for c in range(4):
        for j in range(p.n_theta):
            assert out[c * n + j * nr] == 0 and out[c * n + j * nr + nr - 1] == 0


def test_engine_matches_450bit_scheme_with_full_precision_tables():
    """The engine fed the 450-bit mpmath tables directly (not dyadic-rounded
    ones) agrees with the Python scheme run at 450 bits: pins the conversion
    of wide mpmath numbers into fixed point."""
    p = problem.Problem(s=-2, m=1, a_over_M=0.7, n_r=10, n_theta=7, rstar_min=-5.0, rstar_max=40.0)
    tab = problem.build_tables(p)
    rng = np.random.default_rng(12)
    f = [rng.standard_normal((p.n_theta, p.n_r)) for _ in range(4)]
    for x in f:
        x[:, 0] = x[:, -1] = 0
    out = engine.run_problem(p, f, 2, tables=tab)
    n = p.n_r * p.n_theta
    with mp.workprec(450):
        TP = scheme.as_pairs(tab)
        phi = [[(mp.mpf(f[0][j, i]), mp.mpf(f[1][j, i])) for i in range(p.n_r)] for j in range(p.n_theta)]
        pi = [[(mp.mpf(f[2][j, i]), mp.mpf(f[3][j, i])) for i in range(p.n_r)] for j in range(p.n_theta)]
        phi, pi = scheme.evolve(phi, pi, TP, 2, mp.mpf(1) / 2)
        worst = max(abs(mp.mpf(out[c * n + j * p.n_r + i]) / mp.mpf(2) ** FRAC - arr[j][i][c % 2])
                    for c, arr in enumerate((phi, phi, pi, pi)) for j in range(p.n_theta) for i in range(p.n_r))
        assert worst < mp.mpf(2) ** -360, float(worst)


def test_round_scaled_is_exact_for_wide_numbers():
    with mp.workprec(450):
        x = -mp.pi / 7
        negx = -x
    assert engine.round_scaled(x, 400) == -engine.round_scaled(negx, 400)
    with mp.workprec(900):
        ref = int(mp.nint(mp.ldexp(x, 400)))
    assert engine.round_scaled(x, 400) == ref
    assert engine.round_scaled(Fraction(-3, 8), 2) == -2 and engine.round_scaled(Fraction(5, 8), 2) == 3
