"""Grid, time step and coefficient tables of one Teukolsky problem (test infrastructure).

Readings of the paper (it fixes none of these):

* r* grid: n_r vertex-centred nodes r*_i = r*_min + i h, h = (r*_max - r*_min)/(n_r - 1),
  i = 0..n_r-1; the first and last node carry the Dirichlet condition
  Phi = Pi = 0 (Sec. "Teukolsky Code").  Half points r*_{i+1/2} = r*_i + h/2.
* theta grid: n_theta cell centres theta_j = (j + 1/2) k, k = pi / n_theta,
  so the poles are never grid points; the angular boundary condition is
  imposed through reflected ghost values (see ``scheme``).
* time step: dt = cfl * min(h, k) (k in radians, r* in units of M).
* coefficients of the first-order system are evaluated at the location where
  the Lax-Wendroff stage needs them: at r*_{i+1/2} for the half step (lw1)
  and at r*_i for the full step (lw2).
"""
from dataclasses import dataclass
from fractions import Fraction
import multiprocessing as mproc

import mpmath as mp

from . import kerr
from .stencils import central_weights, angular_reach

COEF_NAMES = ("b", "W", "K", "Ct", "C0")      # K, Ct, C0 complex


@dataclass(frozen=True)
class Problem:
    s: int
    m: int
    a_over_M: float
    n_r: int
    n_theta: int
    rstar_min: float
    rstar_max: float
    cfl: float = 0.5
    mass: float = 1.0
    angular_order: int = 10

    def validate(self):
        if abs(self.s) > 2:
            raise ValueError("|s| <= 2")
        if self.n_theta < 5 or self.n_r < 3 or not self.rstar_min < self.rstar_max or self.cfl <= 0:
            raise ValueError("bad grid")
        if self.mass == 0 and (self.a_over_M != 0 or self.rstar_min <= 0):
            raise ValueError("flat space needs a = 0 and r*_min > 0")
        if not abs(self.a_over_M) < 1:
            raise ValueError("|a/M| < 1")


def _prec():
    return mp.workprec(kerr.WORK_BITS)


def grid_scalars(p: Problem):
    """h, k = dtheta, dt and the node positions as mp numbers."""
    with _prec():
        rmin, rmax = mp.mpf(p.rstar_min), mp.mpf(p.rstar_max)
        h = (rmax - rmin) / (p.n_r - 1)
        k = mp.pi / p.n_theta
        dt = mp.mpf(p.cfl) * min(h, k)
        return {"h": h, "dtheta": k, "dt": dt, "rstar_min": rmin}


def _radial_worker(args):
    rs, M, a = args
    with _prec():
        return kerr.r_of_tortoise(mp.mpf(rs), mp.mpf(M), mp.mpf(a))


def _point_worker(args):
    r, j_list, trig, s, m, M, a = args
    with _prec():
        out = []
        for j in j_list:
            c = kerr.background(r, trig[j][0], trig[j][1], s, m, M, a)
            out.append(tuple(c[n] for n in COEF_NAMES))
        return out


def build_tables(p: Problem, processes: int = 1):
    """All time-independent tables the scheme needs, at WORK_BITS precision.

    Returns a dict:
      half[j][i] = (b, W, K, Ct, C0) at (r*_{i+1/2}, theta_j), i = 0..n_r-2
      full[j][i] = (b, W, K, Ct, C0) at (r*_i, theta_j),       i = 0..n_r-1
      cot[j], V[j]                    angular operator factors
      d1[k], d2[k]                    stencil weights / dtheta, / dtheta^2 (k = -R..R)
      parity                          ghost sign (-1)^|m| (Sec. "Teukolsky Code")
      h, dt, dtheta                   scalars
    """
    p.validate()
    with _prec():
        g = grid_scalars(p)
        M = mp.mpf(p.mass)
        a = mp.mpf(p.a_over_M) * M
        h, k = g["h"], g["dtheta"]
        rs_full = [g["rstar_min"] + i * h for i in range(p.n_r)]
        rs_half = [g["rstar_min"] + (i + mp.mpf(1) / 2) * h for i in range(p.n_r - 1)]
        trig = []
        for j in range(p.n_theta):
            th = (j + mp.mpf(1) / 2) * k
            c, sn = mp.cos(th), mp.sin(th)
            trig.append((c, sn * sn, c / sn))
        jobs = [(x, M, a) for x in rs_full + rs_half]
        if processes > 1:
            with mproc.get_context("fork").Pool(processes) as pool:
                radii = pool.map(_radial_worker, jobs, chunksize=16)
        else:
            radii = [_radial_worker(x) for x in jobs]
        r_full, r_half = radii[:p.n_r], radii[p.n_r:]
        jl = list(range(p.n_theta))
        pjobs = [(r, jl, trig, p.s, p.m, M, a) for r in r_full + r_half]
        if processes > 1:
            with mproc.get_context("fork").Pool(processes) as pool:
                cols = pool.map(_point_worker, pjobs, chunksize=4)
        else:
            cols = [_point_worker(x) for x in pjobs]
        cf, ch = cols[:p.n_r], cols[p.n_r:]
        full = [[cf[i][j] for i in range(p.n_r)] for j in range(p.n_theta)]
        half = [[ch[i][j] for i in range(p.n_r - 1)] for j in range(p.n_theta)]
        R = angular_reach(p.angular_order)
        c1 = central_weights(1, R)
        c2 = central_weights(2, R)
        d1 = [mp.mpf(c.numerator) / c.denominator / k for c in c1]
        d2 = [mp.mpf(c.numerator) / c.denominator / (k * k) for c in c2]
        cot = [t[2] for t in trig]
        V = [kerr.angular_potential(t[0], t[1], p.s, p.m) for t in trig]
        return {"half": half, "full": full, "cot": cot, "V": V, "d1": d1, "d2": d2,
                "reach": R, "parity": -1 if abs(p.m) % 2 else 1,
                "h": h, "inv_h": 1 / h, "dt": g["dt"], "dtheta": k,
                "r_full": r_full, "r_half": r_half}


def to_fractions(tables, bits: int = 120):
    """Round every real table entry to a dyadic rational with ``bits`` fraction bits.

    Used by the exact-arithmetic brute force: the rounded tables define a
    scheme whose exact evolution is computable in Fractions.
    """
    from .engine import round_scaled

    def q(x):
        return Fraction(round_scaled(x, bits), 1 << bits)

    def qc(z):
        if isinstance(z, mp.mpc):
            return (q(z.real), q(z.imag))
        return q(z)

    out = dict(tables)
    for key in ("half", "full"):
        out[key] = [[tuple(qc(v) for v in pt) for pt in row] for row in tables[key]]
    for key in ("cot", "V", "d1", "d2"):
        out[key] = [q(v) for v in tables[key]]
    for key in ("h", "inv_h", "dt", "dtheta"):
        out[key] = q(tables[key])
    return out
