"""Frozen-coefficient amplification of the two Lax-Wendroff stages on the
angular part of the system (TEST INFRASTRUCTURE ONLY: it fixes the reading
of the time step, which the paper does not state).

With the radial derivatives, C_t and K dropped and the coefficients frozen at
one Boyer-Lindquist radius r, the first-order system (Sec. "Teukolsky Code")
reduces on a theta column to

    d_t Phi = Pi,   d_t Pi = A Phi,   A = diag(W(r, theta_j)) L_h,

with L_h the discrete angular operator of the scheme (centred differences,
ghost rows reflected with sign (-1)^|m|) and W = Delta / Sigma^2.  For data
constant along r*, stage (lw1) is u^{n+1/2} = u + (dt/2) B u and stage (lw2)
u^{n+1} = u + dt B u^{n+1/2}, B = [[0, I], [A, 0]], so one step multiplies by
G = I + dt B + (dt B)^2 / 2.  B has the eigenvalues +-sqrt(lambda) for each
eigenvalue lambda of A, so the per-step amplification of that mode is
|1 + mu + mu^2 / 2| with mu = +-dt sqrt(lambda).  For lambda < 0 (mu = i y)
this is sqrt(1 + y^4 / 4) > 1: the explicit midpoint rule's weak growth,
which the stiff pole term (m + s cos)^2 / sin^2 of s = -2 makes large.

The analysis is a bound in the frozen-coefficient sense, not a run; the
eigenvalues are taken in float64 (the matrix entries come from the oracle's
450-bit tables).
"""
import mpmath as mp
import numpy as np

from . import kerr, problem, scheme


def angular_matrix(s: int, m: int, n_theta: int, angular_order: int = 10) -> np.ndarray:
    """L_h as a float64 n_theta x n_theta matrix: column q is the oracle's
    angular operator applied to the q-th unit column."""
    p = problem.Problem(s=s, m=m, a_over_M=0.0, n_r=3, n_theta=n_theta, rstar_min=-1.0, rstar_max=1.0,
                        angular_order=angular_order)
    tab = problem.build_tables(p)
    L = np.zeros((n_theta, n_theta))
    with mp.workprec(kerr.WORK_BITS):
        zero = mp.mpf(0)
        for q in range(n_theta):
            col = [(mp.mpf(1) if j == q else zero, zero) for j in range(n_theta)]
            for j in range(n_theta):
                L[j, q] = float(scheme.theta_operator(col, j, tab)[0])
    return L


def w_column(r: float, n_theta: int, a_over_M: float, M: float = 1.0) -> np.ndarray:
    """W = Delta / Sigma^2 at radius r on the cell-centred theta rows."""
    with mp.workprec(kerr.WORK_BITS):
        a = mp.mpf(a_over_M) * M
        out = []
        for j in range(n_theta):
            th = (j + mp.mpf(1) / 2) * mp.pi / n_theta
            c, sn = mp.cos(th), mp.sin(th)
            out.append(float(kerr.background(mp.mpf(r), c, sn * sn, 0, 0, M, a)["W"]))
    return np.array(out)


def step_factor(lam: np.ndarray, dt: float) -> np.ndarray:
    """Largest |1 + mu + mu^2/2| over mu = +-dt sqrt(lambda), per eigenvalue lambda."""
    mu = dt * np.sqrt(lam.astype(complex))
    g1 = np.abs(1 + mu + mu * mu / 2)
    g2 = np.abs(1 - mu + mu * mu / 2)
    return np.maximum(g1, g2)


def update_matrix(A: np.ndarray, dt: float) -> np.ndarray:
    """The explicit two-stage update of (Phi, Pi) for d_t Phi = Pi, d_t Pi = A Phi."""
    n = A.shape[0]
    B = np.block([[np.zeros((n, n)), np.eye(n)], [A, np.zeros((n, n))]])
    Uh = np.eye(2 * n) + 0.5 * dt * B               # stage (lw1)
    return np.eye(2 * n) + dt * B @ Uh              # stage (lw2)


def worst_amplification(s: int, m: int, a_over_M: float, n_theta: int, h: float, cfl: float,
                        radii=None, L: np.ndarray = None):
    """(max |G| per step, radius where it occurs) over radii outside the
    horizon, with dt = cfl * min(h, pi / n_theta)."""
    if L is None:
        L = angular_matrix(s, m, n_theta)
    dt = cfl * min(h, np.pi / n_theta)
    if radii is None:
        rp = 1.0 + np.sqrt(1.0 - a_over_M ** 2)
        radii = rp + np.concatenate([np.geomspace(1e-3, 1.0, 40), np.linspace(1.05, 12.0, 120)])
    best, where = 0.0, None
    for r in radii:
        lam = np.linalg.eigvals(w_column(r, n_theta, a_over_M)[:, None] * L)
        g = float(step_factor(lam, dt).max())
        if g > best:
            best, where = g, float(r)
    return best, where


def radial_update_matrix(p, processes: int = 1) -> np.ndarray:
    """The oracle's one-step map restricted to real, theta-independent data
    (exact for s = 0, m = 0, a = 0, where such data stay theta-independent
    and real): column q is one step of the fixed-point engine applied to the
    q-th unit vector of (Phi, Pi) at the interior r* nodes, read back on the
    first theta row and rounded to float64."""
    from . import engine
    if not (p.s == 0 and p.m == 0 and p.a_over_M == 0):
        raise ValueError("theta-independent real data are invariant only for s = m = a = 0")
    tab = problem.build_tables(p, processes=processes)
    FT = engine.tables_to_fixed(tab)
    nr, nth = p.n_r, p.n_theta
    interior = list(range(1, nr - 1))
    ni = len(interior)
    U = np.zeros((2 * ni, 2 * ni))
    one = 1 << engine.FRAC
    plane = nr * nth
    for col in range(2 * ni):
        comp, i = (0, interior[col]) if col < ni else (2, interior[col - ni])
        u = [0] * (4 * plane)
        for j in range(nth):
            u[comp * plane + j * nr + i] = one
        out = engine.run_fixed(FT, nr, nth, u, 1)
        for row in range(2 * ni):
            c, k = (0, interior[row]) if row < ni else (2, interior[row - ni])
            U[row, col] = out[c * plane + k] / one
    return U


def radial_spectral_radius(p, processes: int = 1):
    """(largest |eigenvalue| of radial_update_matrix, r* node where its eigenvector peaks)."""
    U = radial_update_matrix(p, processes=processes)
    ev, vec = np.linalg.eig(U)
    k = int(np.argmax(np.abs(ev)))
    ni = U.shape[0] // 2
    i = int(np.argmax(np.abs(vec[:ni, k]))) + 1
    h = (p.rstar_max - p.rstar_min) / (p.n_r - 1)
    return float(np.abs(ev[k])), p.rstar_min + i * h
