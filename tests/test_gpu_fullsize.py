"""GPU parity at full sizes: the workloads' full step counts against oracle
reference data written by tests/golden/make_golden.py (sampled grid points
plus the exact global maximum, which normalises the relative L-infinity), and
the headline grid in every precision against a live oracle run on an r* slab
that holds the domain of dependence of a window around the pulse."""
import glob
import json
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_0663_amd import inputs, teuk as T
from oracle import engine
from parity_util import gpu_ints, to_problem

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = sorted(glob.glob(os.path.join(HERE, "golden", "*.npz")))
TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60}


def _value(words):
    return sum((Fraction(float(x)) for x in words), Fraction(0))


def load(path):
    z = np.load(path, allow_pickle=False)
    w = inputs.Workload(**json.loads(str(z["workload"])))
    return w, z["points"], z["values"], _value(z["maxabs"])


@pytest.mark.parametrize("mode", ["default", "tuned"])
@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f)[:-4] for f in FILES])
def test_full_size_parity(path, mode, tmp_path, monkeypatch):
    """mode "default": the library's launch shape; "tuned": the shape the
    autotuner picks with graphs on, which is how bench.py times a workload
    (fused multi-step launches included)."""
    w, pts, vals, maxabs = load(path)
    print("full-size parity %s (%s launch shape): %dx%d words=%d steps=%d cfl=%g"
          % (w.name, mode, w.n_r, w.n_theta, w.words, w.steps, w.cfl), flush=True)
    g = T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)
    h = T.Teuk(w.s, w.m, w.a_over_M, g, w.words)
    h.use_graph(100)                       # as bench.py times it
    h.set_initial(*inputs.initial_fields(w))
    if mode == "tuned":
        import torch
        from paper_1006_0663_amd import autotune
        monkeypatch.setenv("TEUK_TUNE_CACHE", str(tmp_path / "cache.json"))
        torch.cuda.set_device(0)
        stream = torch.cuda.Stream()
        h.set_stream(stream.cuda_stream)
        shape = autotune.tune(h, w.words, [(w.n_r, w.n_theta)], torch, stream, steps=200)
        print("  tuned shape (sweep, segcols, block, steps per launch, us): %s" % (shape,), flush=True)
        h.set_initial(*inputs.initial_fields(w))
    h.step(w.steps)
    got = [h.read_field(c).reshape(-1, w.words) for c in range(4)]
    h.close()
    worst = Fraction(0)
    for k, q in enumerate(pts):
        for c in range(4):
            worst = max(worst, abs(_value(got[c][q]) - _value(vals[k, c])))
    rel = float(worst / maxabs)
    print("  rel Linf over %d sampled points = %.3e (tolerance %.0e)" % (len(pts), rel, TOL[w.words]), flush=True)
    assert rel <= TOL[w.words]


WINDOW = [inputs.C2, inputs.C2_DD, inputs.C2_QD]


@pytest.mark.parametrize("w", WINDOW, ids=[x.name for x in WINDOW])
def test_headline_grid_window_parity(w, tmp_path, monkeypatch):
    """The whole 4096 x 128 headline grid in each precision, in the launch
    shape the autotuner picks (as bench.py times it), against the oracle on an
    r* slab around the pulse: after n steps a node depends only on nodes within
    n of it, so a slab reaching n + 1 nodes beyond the compared window gives
    the window's exact oracle values (checked on the CPU: identical integers).
    Relative L-infinity over the window, normalised by the window's largest
    reference value (the pulse peak lies inside it)."""
    import mpmath as mp
    import torch
    from oracle import kerr
    from paper_1006_0663_amd import autotune
    n, half = 8, 4
    fields = inputs.initial_fields(w)
    monkeypatch.setenv("TEUK_TUNE_CACHE", str(tmp_path / "cache.json"))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    h = T.Teuk(w.s, w.m, w.a_over_M, T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass,
                                                 w.angular_order), w.words)
    h.set_stream(stream.cuda_stream)
    h.use_graph(100)
    h.set_initial(*fields)
    shape = autotune.tune(h, w.words, [(w.n_r, w.n_theta)], torch, stream, steps=100)
    print("window parity %s: tuned shape %s" % (w.name, shape), flush=True)
    h.set_initial(*fields)
    h.step(n)
    got = [h.read_field(c) for c in range(4)]
    h.close()
    peak = int(abs(fields[0][..., 0]).sum(axis=0).argmax())
    lo, hi = peak - half - n - 1, peak + half + n + 1
    assert 0 < lo and hi < w.n_r - 1
    with mp.workprec(kerr.WORK_BITS):
        hr = (mp.mpf(w.rstar_max) - mp.mpf(w.rstar_min)) / (w.n_r - 1)
        rmin, rmax = mp.mpf(w.rstar_min) + lo * hr, mp.mpf(w.rstar_min) + hi * hr
    ns = hi - lo + 1
    slab = w.with_(n_r=ns)
    out = engine.run_problem(to_problem(slab, rstar_min=rmin, rstar_max=rmax), [f[:, lo:hi + 1] for f in fields],
                             n, processes=16)
    err, mx = 0, 0
    for c in range(4):
        g = gpu_ints(got[c][:, peak - half:peak + half + 1])
        r = [out[c * ns * w.n_theta + j * ns + i] for j in range(w.n_theta)
             for i in range(peak - half - lo, peak + half - lo + 1)]
        err = max(err, max(abs(a - b) for a, b in zip(g, r)))
        mx = max(mx, max(abs(b) for b in r))
    rel = err / mx
    print("  rel Linf over the %d x %d window = %.3e (tolerance %.0e)" % (2 * half + 1, w.n_theta, rel,
                                                                         TOL[w.words]), flush=True)
    assert mx > 0 and rel <= TOL[w.words]


# (workload, higher precision): the same run in more words is within a small
# multiple of its own tolerance of the exact scheme (the sampled points above
# pin the higher-precision runs against the oracle), so the difference bounds
# the lower-precision result's error at every grid point
HIGHER = [(inputs.C2, 2), (inputs.C3_PARITY, 4)]


@pytest.mark.parametrize("w,words_hi", HIGHER, ids=["%s-vs-%dw" % (x[0].name, x[1]) for x in HIGHER])
def test_full_grid_against_higher_precision(w, words_hi):
    """Every point of every field after the workload's full step count, in the
    default launch shape with graphs, against the same workload run in more
    words: rel L-infinity within the lower precision's tolerance."""
    import numpy as np
    print("full grid %s (%d steps) against %d words" % (w.name, w.steps, words_hi), flush=True)
    out = {}
    for words in (w.words, words_hi):
        wx = w.with_(words=words)
        h = T.Teuk(wx.s, wx.m, wx.a_over_M, T.make_grid(wx.n_r, wx.n_theta, wx.rstar_min, wx.rstar_max, wx.cfl,
                                                       wx.mass, wx.angular_order), words)
        h.use_graph(100)
        h.set_initial(*inputs.initial_fields(wx))
        h.step(wx.steps)
        out[words] = [h.read_field(c) for c in range(4)]
        h.close()
    lo, hi = out[w.words], out[words_hi]
    # difference of the word expansions, leading words first: the leading
    # difference is exact (Sterbenz) where the values are close, and each
    # later term adds a rounding error of order 2^-53 of itself, far below
    # the tolerance
    err, mx = 0.0, 0.0
    for c in range(4):
        a = lo[c].reshape(-1, w.words)
        b = hi[c].reshape(-1, words_hi)
        d = a[:, 0] - b[:, 0]
        for k in range(1, words_hi):
            d = d + ((a[:, k] if k < w.words else 0.0) - b[:, k])
        err = max(err, float(np.max(np.abs(d))))
        mx = max(mx, float(np.max(np.abs(b[:, 0]))))
    rel = err / mx
    print("  rel Linf over all %d points = %.3e (tolerance %.0e)" % (w.n_r * w.n_theta, rel, TOL[w.words]),
          flush=True)
    assert rel <= TOL[w.words]
