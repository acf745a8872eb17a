"""GPU parity at the workloads' full sizes and step counts, against oracle
reference data written by tests/golden/make_golden.py (sampled grid points
plus the exact global maximum, which normalises the relative L-infinity)."""
import glob
import json
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_0663_amd import inputs, teuk as T

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
