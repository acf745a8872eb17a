"""Helpers shared by the GPU parity tests: run the oracle and compare."""
import json
from fractions import Fraction

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


def word_value(words) -> Fraction:
    """Exact value of a float64 word expansion."""
    return sum((Fraction(float(x)) for x in words), Fraction(0))


def load_golden(path):
    """(workload, sampled point indices, their values [npts][4][4 words], exact max |value|)
    from a file written by tests/golden/make_golden.py."""
    from paper_1006_0663_amd import inputs
    z = np.load(path, allow_pickle=False)
    w = inputs.Workload(**json.loads(str(z["workload"])))
    return w, z["points"], z["values"], word_value(z["maxabs"])


def golden_rel_err(fields, pts, vals, maxabs):
    """Largest |gpu - oracle| over the sampled points and components, over max |oracle|."""
    got = [np.asarray(f).reshape(-1, np.asarray(f).shape[-1]) for f in fields]
    worst = Fraction(0)
    for k, q in enumerate(pts):
        for c in range(4):
            worst = max(worst, abs(word_value(got[c][q]) - word_value(vals[k, c])))
    return float(worst / maxabs)


def window_parity(w, fields, got, n, half=4, processes=16):
    """Relative L-infinity of a GPU result `got` (4 field arrays after n steps
    from `fields`) over a window of 2 half + 1 r* nodes around the pulse peak,
    against the oracle run on an r* slab that reaches n + 1 nodes beyond the
    window: after n steps a node depends only on nodes within n of it, so the
    slab gives the window's values exactly.  Normalised by the window's
    largest oracle value."""
    import mpmath as mp
    from oracle import kerr
    peak = int(abs(np.asarray(fields[0])[..., 0]).sum(axis=0).argmax())
    lo, hi = peak - half - n - 1, peak + half + n + 1
    assert 0 < lo and hi < w.n_r - 1, "window too close to a radial boundary"
    with mp.workprec(kerr.WORK_BITS):
        hr = (mp.mpf(w.rstar_max) - mp.mpf(w.rstar_min)) / (w.n_r - 1)
        rmin, rmax = mp.mpf(w.rstar_min) + lo * hr, mp.mpf(w.rstar_min) + hi * hr
    ns = hi - lo + 1
    slab = w.with_(n_r=ns)
    out = engine.run_problem(to_problem(slab, rstar_min=rmin, rstar_max=rmax),
                             [np.asarray(f)[:, lo:hi + 1] for f in fields], n, processes=processes)
    err, mx = 0, 0
    for c in range(4):
        g = gpu_ints(np.asarray(got[c])[:, peak - half:peak + half + 1])
        r = [out[c * ns * w.n_theta + j * ns + i] for j in range(w.n_theta)
             for i in range(peak - half - lo, peak + half - lo + 1)]
        err = max(err, max(abs(a - b) for a, b in zip(g, r)))
        mx = max(mx, max(abs(b) for b in r))
    assert mx > 0
    return err / mx
