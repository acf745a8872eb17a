"""GPU checks of the batched form at the size the benchmark times it: the 32
uneven double-double instances (n_r up to 8192, n_theta up to 256), advanced
together in the launch shape the autotuner picks, against single-instance
runs (bitwise) and against the oracle (a window around the pulse of three
instances, and the full step count of the two instances with reference data).
"""
import glob
import os
import sys

import numpy as np
import pytest

from paper_1006_0663_amd import inputs, teuk as T
from parity_util import golden_rel_err, load_golden, window_parity

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_DD = 1e-28


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _grid(w):
    return T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)


def _single(w, fields, nsteps):
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), w.words)
    h.set_initial(*fields)
    h.step(nsteps)
    out = h.fields()
    h.close()
    return out


@pytest.fixture(scope="module")
def c5():
    ws = inputs.batch_workloads()
    _note("generating the 32 batched instances")
    return ws, [inputs.initial_fields(w) for w in ws]


def test_timed_batch_shape_equals_single_and_oracle(c5, tmp_path, monkeypatch):
    """All 32 instances in one batch, in the autotuned shape with graph
    replay, 8 steps: every instance equals its own single-instance run
    (default shape) bit for bit, and three of them (the two 8192 x 256
    instances with m = 4, one of them a/M = 0.958, and the smallest) match the
    oracle on a window around the pulse."""
    import torch
    from paper_1006_0663_amd import autotune
    ws, fields = c5
    monkeypatch.setenv("TEUK_TUNE_CACHE", str(tmp_path / "cache.json"))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 2)
    b.set_stream(stream.cuda_stream)
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    shape = autotune.tune(b, 2, [(w.n_r, w.n_theta) for w in ws], torch, stream, steps=8, reps=1)
    _note("batch of 32: tuned shape %s" % (shape,))
    b.use_graph(4)
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    n = 8
    b.step(n)
    assert b.graph_replays >= 1
    check = {30, 9, 5}
    for k, w in enumerate(ws):
        got = [b.read_field(k, c) for c in range(4)]
        ref = _single(w, fields[k], n)
        for c in range(4):
            assert np.array_equal(got[c], ref[c]), (k, c)
        if k in check:
            rel = window_parity(w, fields[k], got, n)
            _note("  instance %d (%dx%d m=%d a=%.3f): window rel Linf %.3e" % (k, w.n_r, w.n_theta, w.m,
                                                                               w.a_over_M, rel))
            assert rel <= TOL_DD
    b.close()


def test_golden_instances_in_a_mixed_batch():
    """The two batch instances with full-length oracle reference data, in one
    batch with two large ones (8192 x 256 and 4096 x 128), for the full 2,000
    steps with graph replay: the golden instances match the oracle on the
    sampled points, the large ones equal their single-instance runs."""
    gold = {}
    for path in sorted(glob.glob(os.path.join(HERE, "golden", "batch*.npz"))):
        w, pts, vals, mx = load_golden(path)
        gold[w.name] = (w, pts, vals, mx)
    assert len(gold) == 2
    ws_all = {w.name: w for w in inputs.batch_workloads()}
    for name, (w, *_) in gold.items():
        assert ws_all[name] == w, name
    ws = [gold[k][0] for k in sorted(gold)] + [ws_all["batch30"], ws_all["batch2"]]
    steps = ws[0].steps
    _note("mixed batch %s, %d steps" % ([(w.name, w.n_r, w.n_theta) for w in ws], steps))
    fields = [inputs.initial_fields(w) for w in ws]
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 2)
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    b.use_graph(100)
    b.step(steps)
    assert b.graph_replays == steps // 100          # one step per launch by default
    for k, w in enumerate(ws):
        got = [b.read_field(k, c) for c in range(4)]
        if w.name in gold:
            _, pts, vals, mx = gold[w.name]
            rel = golden_rel_err(got, pts, vals, mx)
            _note("  %s: rel Linf over %d sampled points %.3e" % (w.name, len(pts), rel))
            assert rel <= TOL_DD
        else:
            ref = _single(w, fields[k], steps)
            for c in range(4):
                assert np.array_equal(got[c], ref[c]), (w.name, c)
    b.close()
