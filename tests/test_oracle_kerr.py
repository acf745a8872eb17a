"""Pins of oracle.kerr against Eq. (1) of the paper, closed forms and limits."""
import random

import mpmath as mp
import pytest

from oracle import kerr


def _eq1_residual(s, m, a, t, r, th, M=1):
    """Relative residual of Eq. (1) for Psi = exp(i m phi~) r^3 Phi, with Phi
    the solution of the oracle's first-order system written as a second-order
    equation; all derivatives of Psi by numerical differentiation."""
    M = mp.mpf(M)
    a = mp.mpf(a)
    rp, rm = kerr.horizons(M, a)
    al, be, ga = mp.mpc("0.3", "0.7"), mp.mpc("-0.11", "0.23"), mp.mpc("0.4", "-0.2")
    I = mp.mpc(0, 1)

    def Phi(t, x, th):
        return mp.exp(al * t + be * x + ga * mp.cos(th))

    def g(r):                           # phi~ - phi = int a/Delta dr
        return a / (rp - rm) * mp.log((r - rp) / (r - rm)) if a != 0 else mp.mpf(0)

    def Psi(t, r, th):
        return mp.exp(I * m * g(r)) * r ** 3 * Phi(t, kerr.tortoise(r, M, a), th)

    delta, varpi = r * r - 2 * M * r + a * a, r * r + a * a
    sth, cth = mp.sin(th), mp.cos(th)
    D = lambda n: mp.diff(Psi, (t, r, th), n)
    P, Pt, Ptt, Pr, Prr, Pth, Pthth = (D(n) for n in ((0, 0, 0), (1, 0, 0), (2, 0, 0), (0, 1, 0),
                                                     (0, 2, 0), (0, 0, 1), (0, 0, 2)))
    # Eq. (1) with d_phi -> i m
    E = (-(varpi ** 2 / delta - a * a * sth ** 2) * Ptt - 4 * M * a * r / delta * (I * m) * Pt
         - 2 * s * (r - M * (r * r - a * a) / delta + I * a * cth) * Pt
         + delta * Prr + (s + 1) * 2 * (r - M) * Pr + Pthth + cth / sth * Pth
         + (1 / sth ** 2 - a * a / delta) * (-m * m) * P
         + 2 * s * (a * (r - M) / delta + I * cth / sth ** 2) * (I * m) * P
         - (s * s * cth ** 2 / sth ** 2 - s) * P)
    x = kerr.tortoise(r, M, a)
    c = kerr.background(r, cth, sth ** 2, s, m, M, a)
    ph = Phi(t, x, th)
    pht, phx = al * ph, be * ph
    phth = -ga * sth * ph
    phthth = (ga * ga * sth ** 2 - ga * cth) * ph
    lth = phthth + cth / sth * phth + kerr.angular_potential(cth, sth ** 2, s, m) * ph
    b = c["b"]
    bx = mp.diff(lambda rr: kerr.background(rr, cth, sth ** 2, s, m, M, a)["b"], r) * delta / varpi
    Pi = pht + b * phx
    Pit, Pix = al * Pi, be * Pi + bx * phx
    resid = Pit - b * Pix - (-c["K"] * phx + c["W"] * lth + c["C0"] * ph - c["Ct"] * Pi)
    return abs(E + c["Sigma2"] / delta * r ** 3 * mp.exp(I * m * g(r)) * resid) / abs(E)


def test_first_order_system_reproduces_eq1():
    random.seed(11)
    with mp.workprec(300):
        for _ in range(8):
            s = random.choice([-2, -1, 0, 1, 2])
            m = random.randint(-4, 4)
            a = mp.mpf(random.random() * 0.99)
            r = mp.mpf(2.2 + random.random() * 20)
            th = mp.mpf(0.15 + random.random() * 2.8)
            assert _eq1_residual(s, m, a, mp.mpf("0.3"), r, th) < mp.mpf(10) ** -60


def test_planted_sign_error_is_caught(monkeypatch):
    """The identity above must fail for a coefficient with a flipped term."""
    orig = kerr.background

    def wrong(*args):
        c = orig(*args)
        c["C0"] = mp.conj(c["C0"])
        return c
    monkeypatch.setattr(kerr, "background", wrong)
    with mp.workprec(300):
        assert _eq1_residual(-2, 2, mp.mpf("0.6"), mp.mpf("0.3"), mp.mpf(5), mp.mpf(1)) > 1e-6


def test_tortoise_inversion_and_schwarzschild_form():
    with mp.workprec(450):
        for a in ("0", "0.5", "0.99"):
            for rs in ("-200", "-3", "0", "7.5", "800"):
                aa = mp.mpf(a)
                r = kerr.r_of_tortoise(mp.mpf(rs), 1, aa)
                # a residual in r of one unit in the last place moves r* by dr*/dr = varpi/Delta
                cond = (r * r + aa * aa) / (r * r - 2 * r + aa * aa)
                assert abs(kerr.tortoise(r, 1, aa) - mp.mpf(rs)) < mp.mpf(2) ** -400 * (1 + abs(r)) * cond
        # a = 0: r* = r + 2M ln(r/2M - 1) (textbook Regge-Wheeler tortoise coordinate)
        r = mp.mpf("3.7")
        assert abs(kerr.tortoise(r, 1, 0) - (r + 2 * mp.log(r / 2 - 1))) < mp.mpf(2) ** -440
        # dr*/dr = (r^2 + a^2)/Delta
        a = mp.mpf("0.7")
        d = mp.diff(lambda x: kerr.tortoise(x, 1, a), r)
        assert abs(d - (r * r + a * a) / (r * r - 2 * r + a * a)) < mp.mpf(10) ** -100


def test_bdb_closed_form_is_b_times_radial_derivative():
    with mp.workprec(300):
        a, th = mp.mpf("0.9"), mp.mpf("1.1")
        c, s2 = mp.cos(th), mp.sin(th) ** 2
        for r in (mp.mpf("1.9"), mp.mpf("4"), mp.mpf("30")):
            co = kerr.background(r, c, s2, -2, 2, 1, a)
            delta, varpi = r * r - 2 * r + a * a, r * r + a * a
            db = mp.diff(lambda x: kerr.background(x, c, s2, -2, 2, 1, a)["b"], r) * delta / varpi
            assert abs(co["b"] * db - co["bdb"]) < mp.mpf(10) ** -80


@pytest.mark.parametrize("r", ["2.5", "7", "40"])
def test_flat_and_schwarzschild_limits(r):
    with mp.workprec(300):
        r = mp.mpf(r)
        th = mp.mpf("0.8")
        c, s2 = mp.cos(th), mp.sin(th) ** 2
        f = kerr.background(r, c, s2, 0, 3, 0, 0)          # flat space, s = 0
        assert f["b"] == 1 and abs(f["W"] - 1 / r ** 2) < 1e-80
        assert abs(f["Ct"]) < 1e-80 and abs(f["K"] + 8 / r) < 1e-80 and abs(f["C0"] - 12 / r ** 2) < 1e-80
        for s in (-2, 1):
            sch = kerr.background(r + 2, c, s2, s, 2, 1, 0)  # Schwarzschild: every coefficient real
            rr = r + 2
            assert abs(sch["b"] - 1) < 1e-80
            assert abs(sch["Ct"] - 2 * s * (rr - 3) / rr ** 2) < 1e-80
            for k in ("K", "Ct", "C0"):
                assert sch[k].imag == 0
