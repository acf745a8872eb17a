"""Helpers shared by the GPU parity tests: run the oracle and compare."""
import numpy as np

from oracle import engine, problem


def to_problem(w, **over):
    kw = dict(s=w.s, m=w.m, a_over_M=w.a_over_M, n_r=w.n_r, n_theta=w.n_theta, rstar_min=w.rstar_min,
              rstar_max=w.rstar_max, cfl=w.cfl, mass=w.mass, angular_order=w.angular_order)
    kw.update(over)
    return problem.Problem(**kw)


def oracle_run(w, fields, nsteps, processes=1, tables=None):
    """Oracle result as four lists of ints (2^-384 units), each [n_theta*n_r]."""
    out = engine.run_problem(to_problem(w), fields, nsteps, processes=processes, tables=tables)
    n = w.n_r * w.n_theta
    return [out[c * n:(c + 1) * n] for c in range(4)]


def gpu_ints(field):
    """float64 word array [n_theta][n_r][p] -> list of ints (exact word sums, 2^-384 units)."""
    a = np.asarray(field)
    return [engine.words_to_fixed(x) for x in a.reshape(-1, a.shape[-1])]


def rel_linf(gpu_fields, ref):
    """max over components and points of |gpu - ref| / max |ref| (float)."""
    err, mx = 0, 0
    for f, r in zip(gpu_fields, ref):
        g = gpu_ints(f)
        err = max(err, max(abs(a - b) for a, b in zip(g, r)))
        mx = max(mx, max(abs(b) for b in r))
    return err / mx if mx else float(err)
