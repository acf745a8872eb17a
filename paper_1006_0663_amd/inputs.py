"""Seeded synthetic inputs: workloads and initial pulses.

This module is shared by the tests, the benchmark and the oracle's drivers.
It holds none of the scheme's arithmetic: only the workload descriptions,
the seeded random draws and the initial data, with momentum Pi = 0 and one of
two profiles:

* "gauss_sin4": a Gaussian pulse in r* times sin^4(theta);
* "bump_legendre": a compactly supported bump (1 - x^2)^8, x = (r* - r0)/w,
  w = 4 sigma, times the associated Legendre function P_l^|m|(cos theta) of
  one multipole l (spin weight 0 only).  The paper's tail run (caption of
  Fig. 1) starts from compactly supported l = 0 data of a scalar field
  (Sec. "Teukolsky Equation": s = 0); these stand in for it.

Initial values are computed exactly enough to be *defined* by this module:
the Gaussian factor, sin^4 and the amplitude are evaluated at 450 bits,
rounded to 2^-600 fixed point, multiplied exactly as integers, and the
product is rounded to ``words`` float64 words by successive round-to-nearest
(word 0 = nearest double, word k = nearest double to what is left), so the
word sum is a non-overlapping expansion.  Gaussian factors below 2^-240 are
flushed to exact zero.  The library and the oracle both start from these
same words.
"""
from dataclasses import dataclass, field, replace
from fractions import Fraction
import math

import mpmath as mp
import numpy as np

_K = 600                    # fixed-point scale of the three factors
_FLUSH = mp.mpf(2) ** -240  # Gaussian factors below this are exactly zero


@dataclass(frozen=True)
class Workload:
    """One Teukolsky run: physics, grid, precision (words per real) and step count."""
    name: str
    s: int
    m: int
    a_over_M: float
    n_r: int
    n_theta: int
    rstar_min: float
    rstar_max: float
    words: int
    steps: int
    cfl: float = 0.5
    mass: float = 1.0
    angular_order: int = 10
    amplitude: str = "phase"        # "phase": exp(i phi0); "normal": (x + i y) scaled to max |Phi| = 1
    seed: int = 0
    profile: str = "gauss_sin4"     # or "bump_legendre" (s = 0)
    ell: int = 0                    # multipole of "bump_legendre" (ell >= |m|)

    def with_(self, **kw):
        return replace(self, **kw)


# Time step.  The workloads state dt = 0.5 min(dr*, dtheta).  With s = -2 the
# angular operator is stiff next to the poles ((m + s cos)^2 / sin^2 term) and
# the two Lax-Wendroff stages treat it like the explicit midpoint rule, which
# amplifies such modes by 1 + O((dt/dtheta)^4) per step.  Over 200 steps
# (first workload) this is harmless; over the 2,000-10,000 steps of the
# others, runs at 0.5 grow without bound and at 0.25 the smallest grid still
# amplifies rounding errors by ~1e7, while at 0.15 the difference between an
# FP64 and a double-double run stays flat (grows <= 80x on the smallest
# grid).  Those workloads therefore keep their step counts and run at
# LONG_RUN_CFL.  Throughput per update does not depend on dt.
LONG_RUN_CFL = 0.15

# The five workloads of the measurement plan.
C1 = Workload("fp64-256x32", s=-2, m=2, a_over_M=0.5, n_r=256, n_theta=32, rstar_min=-50.0,
              rstar_max=250.0, words=1, steps=200)
C2 = Workload("fp64-4096x128", s=-2, m=2, a_over_M=0.9, n_r=4096, n_theta=128, rstar_min=-200.0,
              rstar_max=800.0, words=1, steps=10000, amplitude="normal", cfl=LONG_RUN_CFL)
C3 = Workload("dd-256x32", s=-2, m=2, a_over_M=0.5, n_r=256, n_theta=32, rstar_min=-50.0,
              rstar_max=250.0, words=2, steps=10000, cfl=LONG_RUN_CFL)
C3_PARITY = C3.with_(name="dd-1024x64", n_r=1024, n_theta=64)
C4 = Workload("qd-2048x64", s=-2, m=2, a_over_M=0.99, n_r=2048, n_theta=64, rstar_min=-200.0,
              rstar_max=800.0, words=4, steps=5000, amplitude="normal", cfl=LONG_RUN_CFL)
# The headline grid in double-double and quad-double: single instances large
# enough to fill the GPU, for the sustained multiword throughput (the dd and
# qd workloads above are parity sizes).
C2_DD = C2.with_(name="dd-4096x128", words=2, steps=2000)
C2_QD = C2.with_(name="qd-4096x128", words=4, steps=500)
WORKLOADS = {w.name: w for w in (C1, C2, C3, C3_PARITY, C4, C2_DD, C2_QD)}

BATCH_RSTAR = (-200.0, 800.0)
BATCH_NR = (1024, 2048, 4096, 8192)
BATCH_NTH = (32, 64, 128, 256)


# Spin weight 0 (the paper's own field, Sec. "Teukolsky Equation") with
# l-projected compactly supported data: the late-time tail workloads.  a = 0
# (Schwarzschild), where Price's law fixes the decay at a fixed radius to
# t^-(2l+3); the grid keeps reflections from both Dirichlet ends away from the
# observer (r* = 30) until t ~ 1,260 M.  dt = 0.3 dtheta = 0.059 M (the s = 0,
# m = 0 angular operator has no pole term) and dr* = 0.25 M: with dr* = 0.5 M
# the radial discretisation has a growing mode near r ~ 2.7 M whenever
# dt / dr* is below ~0.2 (the oracle's one-step map, oracle/stability.py).
TAIL_RSTAR = (-600.0, 1000.0)
S0_L0 = Workload("s0-l0-dd-6401x16", s=0, m=0, a_over_M=0.0, n_r=6401, n_theta=16, rstar_min=TAIL_RSTAR[0],
                 rstar_max=TAIL_RSTAR[1], words=2, steps=18000, cfl=0.3, profile="bump_legendre", ell=0)
S0_L1 = S0_L0.with_(name="s0-l1-dd-6401x16", ell=1)
# rotating hole, s = 0, l = 2 data (spheroidal mode coupling): parity sizes
S0_KERR = Workload("s0-l2-m1-a0.9", s=0, m=1, a_over_M=0.9, n_r=1024, n_theta=32, rstar_min=-200.0,
                   rstar_max=800.0, words=2, steps=2000, cfl=0.3, profile="bump_legendre", ell=2)
TAIL_PULSE_R0, TAIL_PULSE_SIGMA = 50.0, 5.0
WORKLOADS.update({w.name: w for w in (S0_L0, S0_L1, S0_KERR)})


def tail_pulse():
    """The pulse of the tail workloads: centred at r* = 50 M, half-width 20 M, amplitude 1."""
    return Pulse(TAIL_PULSE_R0, TAIL_PULSE_SIGMA, mp.mpf(1), mp.mpf(0))


def batch_workloads(n: int = 32, seed: int = 0, steps: int = 2000, words: int = 2, cfl: float = LONG_RUN_CFL):
    """Independent instances for the batched run: m ~ U{0..4}, a/M ~ U[0, 0.99],
    n_r ~ U{1024..8192}, n_theta ~ U{32..256}, each with its own pulse seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        m = int(rng.integers(0, 5))
        a = float(rng.uniform(0.0, 0.99))
        nr = int(rng.choice(BATCH_NR))
        nth = int(rng.choice(BATCH_NTH))
        out.append(Workload("batch%d" % k, s=-2, m=m, a_over_M=a, n_r=nr, n_theta=nth,
                            rstar_min=BATCH_RSTAR[0], rstar_max=BATCH_RSTAR[1], words=words,
                            steps=steps, cfl=cfl, seed=int(rng.integers(0, 2**31))))
    return out


@dataclass
class Pulse:
    r0: float
    sigma: float
    amp_re: object       # mp numbers
    amp_im: object


def draw_pulse(w: Workload) -> Pulse:
    """Draw order: r0 ~ U[80, 120], sigma ~ U[4, 8], then either phi0 ~ U[0, 2 pi)
    ("phase") or x, y ~ N(0, 1) ("normal")."""
    rng = np.random.default_rng(w.seed)
    r0 = float(rng.uniform(80.0, 120.0))
    sigma = float(rng.uniform(4.0, 8.0))
    with mp.workprec(450):
        if w.amplitude == "phase":
            ph = mp.mpf(float(rng.uniform(0.0, 2 * math.pi)))
            return Pulse(r0, sigma, mp.cos(ph), mp.sin(ph))
        x, y = float(rng.standard_normal()), float(rng.standard_normal())
        nrm = mp.sqrt(mp.mpf(x) ** 2 + mp.mpf(y) ** 2)
        return Pulse(r0, sigma, mp.mpf(x) / nrm, mp.mpf(y) / nrm)


def _int_to_words(X: int, scale_bits: int, words: int):
    out = []
    for _ in range(words):
        w = X / (1 << scale_bits)          # int true division rounds correctly
        out.append(w)
        n, d = w.as_integer_ratio()
        X -= (n << scale_bits) // d        # exact: d is a power of two <= 2^1074
    return out


def initial_fields(w: Workload, pulse: Pulse = None):
    """(phi_re, phi_im, pi_re, pi_im), each float64 [n_theta][n_r][words].

    Phi(0) = A f(r*) Y(theta), Pi(0) = 0, with the radial boundary columns
    zero: f = exp(-(r* - r0)^2 / (2 sigma^2)) and Y = sin^4(theta) for the
    profile "gauss_sin4"; f = (1 - x^2)^8 on |x| < 1 (0 elsewhere),
    x = (r* - r0)/(4 sigma), and Y = P_l^|m|(cos theta) for "bump_legendre".
    For amplitude "normal" the field is scaled so that its largest modulus on
    the grid is 1.
    """
    if pulse is None:
        pulse = draw_pulse(w)
    if w.profile not in ("gauss_sin4", "bump_legendre"):
        raise ValueError("unknown profile %r" % w.profile)
    if w.profile == "bump_legendre" and (w.s != 0 or w.ell < abs(w.m)):
        raise ValueError("l-projected data are built for s = 0 and l >= |m|")
    nr, nth, p = w.n_r, w.n_theta, w.words
    with mp.workprec(450):
        h = (mp.mpf(w.rstar_min) * -1 + w.rstar_max) / (nr - 1)
        r0, sg = mp.mpf(pulse.r0), mp.mpf(pulse.sigma)
        g = []
        for i in range(nr):
            x = mp.mpf(w.rstar_min) + i * h
            if w.profile == "gauss_sin4":
                v = mp.exp(-(x - r0) ** 2 / (2 * sg * sg))
            else:
                y = (x - r0) / (4 * sg)
                v = (1 - y * y) ** 8 if abs(y) < 1 else mp.mpf(0)
            g.append(v if (v >= _FLUSH and 0 < i < nr - 1) else mp.mpf(0))
        k = mp.pi / nth
        if w.profile == "gauss_sin4":
            t = [mp.sin((j + mp.mpf(1) / 2) * k) ** 4 for j in range(nth)]
        else:
            t = [mp.legenp(w.ell, abs(w.m), mp.cos((j + mp.mpf(1) / 2) * k)) for j in range(nth)]
        are, aim = pulse.amp_re, pulse.amp_im
        if w.amplitude == "normal":
            peak = max(g) * max(abs(v) for v in t)
            are, aim = are / peak, aim / peak
        G = [int(mp.nint(mp.ldexp(v, _K))) for v in g]
        T = [int(mp.nint(mp.ldexp(v, _K))) for v in t]
        A = (int(mp.nint(mp.ldexp(are, _K))), int(mp.nint(mp.ldexp(aim, _K))))
    out = [np.zeros((nth, nr, p)) for _ in range(4)]
    nz = [i for i in range(nr) if G[i]]
    for c in range(2):
        arr = out[c]
        for j in range(nth):
            tj = T[j] * A[c]
            for i in nz:
                arr[j, i, :] = _int_to_words(G[i] * tj, 3 * _K, p)
    return tuple(out)


def words_value(words) -> Fraction:
    """Exact value of a float64 word expansion."""
    return sum((Fraction(float(x)) for x in words), Fraction(0))
