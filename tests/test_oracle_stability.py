"""Pins of the time-step reading (the paper states no time step): the
oracle's frozen-coefficient amplification of the two Lax-Wendroff stages on
the angular part, checked against the explicit two-stage update matrix and
the textbook midpoint-rule factor, its angular operator against the closed-
form eigenfunctions of the s = 0 operator, and the growth it predicts for
the long workloads at the stated CFL 0.5 and at the adopted CFL 0.15."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import stability as S


def test_step_factor_is_the_spectral_radius_of_the_two_stage_update():
    rng = np.random.default_rng(3)
    for n in (3, 6, 9):
        A = rng.standard_normal((n, n)) - 4 * np.eye(n)
        for dt in (0.05, 0.3, 0.9):
            lam = np.linalg.eigvals(A)
            rho = max(abs(np.linalg.eigvals(S.update_matrix(A, dt))))
            assert abs(S.step_factor(lam, dt).max() - rho) <= 1e-10 * rho, (n, dt)


def test_midpoint_rule_factor_for_oscillating_modes():
    # lambda = -omega^2: mu = i y, |G|^2 = 1 + y^4 / 4 (explicit midpoint rule)
    for omega, dt in ((1.0, 0.1), (7.0, 0.05), (30.0, 0.02)):
        y = omega * dt
        g = S.step_factor(np.array([-omega ** 2]), dt)[0]
        assert abs(g * g - (1 + y ** 4 / 4)) <= 1e-13


@pytest.mark.parametrize("m", [0, 1, 2])
def test_angular_matrix_has_the_legendre_eigenvalues(m):
    """s = 0: L = d_thth + cot d_th - m^2 / sin^2 has the eigenfunctions
    P_l^m(cos theta) with eigenvalue -l(l+1); the oracle's discrete operator
    reproduces them to its truncation error, shrinking ~2^-9 per halving."""
    errs = []
    for nth in (24, 48):
        L = S.angular_matrix(0, m, nth)
        th = [(j + mp.mpf(1) / 2) * mp.pi / nth for j in range(nth)]
        worst = 0.0
        for ell in range(m, m + 4):
            v = np.array([float(mp.legenp(ell, m, mp.cos(t))) for t in th])
            res = L @ v + ell * (ell + 1) * v
            worst = max(worst, float(np.abs(res).max() / np.abs(v).max()))
        errs.append(worst)
    assert errs[1] < 1e-6, errs
    assert math.log2(errs[0] / errs[1]) > 8.0, errs


# (s, m, a/M, n_theta, dr*, steps): the FP64 headline, the quad-double
# workload and the worst batched instance (m = 4, a/M = 0.958, 8192 x 256)
LONG = [("fp64-4096x128", -2, 2, 0.9, 128, 1000.0 / 4095, 10000),
        ("qd-2048x64", -2, 2, 0.99, 64, 1000.0 / 2047, 5000),
        ("batch30", -2, 4, 0.958, 256, 1000.0 / 8191, 2000)]


@pytest.mark.parametrize("name,s,m,a,nth,h,steps", LONG, ids=[x[0] for x in LONG])
def test_long_runs_grow_at_cfl_half_and_not_at_0p15(name, s, m, a, nth, h, steps):
    """At the workloads' stated CFL 0.5 the angular pole modes near r ~ 2.5 M
    grow by more than 1e100 over the run; at CFL 0.15 by less than 200."""
    L = S.angular_matrix(s, m, nth)
    rp = 1.0 + math.sqrt(1.0 - a * a)
    radii = rp + np.concatenate([np.geomspace(1e-3, 0.3, 8), np.linspace(0.35, 3.0, 40)])
    g5, r5 = S.worst_amplification(s, m, a, nth, h, 0.5, radii=radii, L=L)
    g15, r15 = S.worst_amplification(s, m, a, nth, h, 0.15, radii=radii, L=L)
    print("%s: CFL 0.5 |G| = %.5f at r = %.3f (|G|^N = %.2e); CFL 0.15 |G| = %.6f (|G|^N = %.2e)"
          % (name, g5, r5, g5 ** steps, g15, g15 ** steps))
    assert steps * math.log10(g5) > 100
    assert g15 ** steps < 200
    assert 2.0 < r5 < 3.2


def _radial(h, dt):
    from oracle import problem
    n = int(round(60.0 / h)) + 1
    k = math.pi / 5
    return problem.Problem(s=0, m=0, a_over_M=0.0, n_r=n, n_theta=5, rstar_min=-20.0, rstar_max=40.0,
                           cfl=dt / min(h, k))


def test_tail_grid_is_radially_stable_and_a_coarser_one_is_not():
    """The oracle's one-step map on theta-independent s = 0 data (exact: such
    data stay theta-independent) around the hole, r* in [-20, 40]: with the
    tail workloads' dt = 0.059 M and dr* = 0.25 M every mode is damped; with
    dr* = 0.5 M (dt / dr* = 0.12) a mode near r ~ 2.7 M (r* ~ 0) grows by
    0.65 % per step, which is what made a first choice of the tail grid blow
    up.  At dt / dr* = 0.5 the coarse grid is stable again."""
    g, where = S.radial_spectral_radius(_radial(0.25, 0.0589), processes=8)
    print("dr* 0.25, dt 0.0589: spectral radius %.8f" % g)
    assert g <= 1.0
    g, where = S.radial_spectral_radius(_radial(0.5, 0.0589), processes=8)
    print("dr* 0.5, dt 0.0589: spectral radius %.8f, mode at r* = %.1f" % (g, where))
    assert g > 1.004 and -5.0 < where < 5.0
    g, _ = S.radial_spectral_radius(_radial(0.5, 0.25), processes=8)
    assert g <= 1.0
