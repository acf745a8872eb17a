"""GPU parity of the hot path against the oracle (small grids: several r*
segments plus a ragged tail, every precision), and the bitwise invariants of
the library (batched == single, checkpoint restart, graph replay, round trip)."""
import sys

import mpmath as mp
import numpy as np
import pytest

from paper_1006_0663_amd import inputs, teuk as T
from oracle import engine, problem
from parity_util import oracle_run, rel_linf, to_problem

pytestmark = pytest.mark.gpu

TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60}


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _grid(w):
    return T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)


def _run_gpu(w, fields, nsteps, tile=None, sweep=None, block=0):
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), w.words)
    if sweep is not None:
        h.set_sweep(sweep)
    if tile:
        h.set_launch(tile, block)
    h.set_initial(*fields)
    h.step(nsteps)
    out = h.fields()
    h.close()
    return out


SMALL = [
    ("flat-s0-m1", inputs.C1.with_(n_r=41, n_theta=10, rstar_min=80.0, rstar_max=130.0, s=0, m=1, a_over_M=0.0,
                                   mass=0.0, words=2)),
    # (label, workload)  -- pulses moved inside the short domains
    ("fp64-m2", inputs.C1.with_(n_r=61, n_theta=16, rstar_min=60.0, rstar_max=150.0, words=1)),
    ("fp64-m1-a0.9", inputs.C1.with_(n_r=45, n_theta=12, rstar_min=70.0, rstar_max=140.0, m=1, a_over_M=0.9, words=1)),
    ("fp64-order2", inputs.C1.with_(n_r=37, n_theta=9, rstar_min=70.0, rstar_max=140.0, angular_order=2, words=1)),
    ("dd-m2", inputs.C1.with_(n_r=61, n_theta=16, rstar_min=60.0, rstar_max=150.0, words=2)),
    ("dd-m3-a0.99", inputs.C4.with_(n_r=45, n_theta=12, rstar_min=60.0, rstar_max=150.0, m=3, words=2)),
    ("qd-m2-a0.99", inputs.C4.with_(n_r=45, n_theta=12, rstar_min=60.0, rstar_max=150.0, words=4)),
    ("qd-m0-a0.3", inputs.C1.with_(n_r=37, n_theta=8, rstar_min=70.0, rstar_max=140.0, m=0, a_over_M=0.3, words=4)),
    # the other spin weights and negative m (every |s| <= 2 and any m are valid)
    ("fp64-s-1-m-1", inputs.C1.with_(n_r=45, n_theta=12, rstar_min=70.0, rstar_max=140.0, s=-1, m=-1,
                                     a_over_M=0.7, words=1)),
    ("fp64-s2-m-2", inputs.C1.with_(n_r=41, n_theta=16, rstar_min=70.0, rstar_max=140.0, s=2, m=-2,
                                    a_over_M=0.9, words=1)),
    ("dd-s1-m-2", inputs.C1.with_(n_r=45, n_theta=12, rstar_min=70.0, rstar_max=140.0, s=1, m=-2,
                                  a_over_M=0.95, words=2)),
    ("dd-s-1-m3", inputs.C1.with_(n_r=39, n_theta=10, rstar_min=70.0, rstar_max=140.0, s=-1, m=3,
                                  a_over_M=0.4, words=2)),
    ("qd-s2-m-3", inputs.C1.with_(n_r=41, n_theta=12, rstar_min=70.0, rstar_max=140.0, s=2, m=-3,
                                  a_over_M=0.5, words=4)),
    ("qd-s1-m-1", inputs.C1.with_(n_r=37, n_theta=8, rstar_min=70.0, rstar_max=140.0, s=1, m=-1,
                                  a_over_M=0.99, words=4)),
]


@pytest.mark.parametrize("sweep", [T.SWEEP_SEGMENT, T.SWEEP_WIDE, T.SWEEP_WIDE2], ids=["segment", "wide", "wide2"])
@pytest.mark.parametrize("label,w", SMALL, ids=[x[0] for x in SMALL])
def test_small_grid_parity(label, w, sweep):
    if sweep == T.SWEEP_WIDE2 and w.words != 1:
        pytest.skip("runs of two columns are built for FP64 only")
    nsteps = 24
    fields = inputs.initial_fields(w)
    _note("parity %s sweep %d: %dx%d words=%d steps=%d" % (label, sweep, w.n_r, w.n_theta, w.words, nsteps))
    got = _run_gpu(w, fields, nsteps, tile=8, sweep=sweep)
    ref = oracle_run(w, fields, nsteps)
    err = rel_linf(got, ref)
    _note("  rel Linf = %.3e (tolerance %.0e)" % (err, TOL[w.words]))
    assert err <= TOL[w.words]


@pytest.mark.parametrize("words", [1, 2, 4])
def test_coefficients_match_oracle(words):
    """Coefficient pass against the oracle's 450-bit Kerr factors, including
    nodes next to the horizon (r* = -200) and far out (r* = 800)."""
    w = inputs.C2.with_(n_r=21, n_theta=8, words=words, a_over_M=0.9, m=3)
    _note("coefficients words=%d" % words)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), words)
    got = [h.coefficients(0), h.coefficients(1)]
    h.close()
    tab = problem.build_tables(to_problem(w))
    with mp.workprec(450):
        scal = {0: (tab["dt"] / 2, tab["dt"] / 2 / tab["h"]), 1: (tab["dt"], tab["dt"] / tab["h"])}
        report = []
        for which, key in ((0, "half"), (1, "full")):
            s, si = scal[which]
            for c in range(8):
                worst, mx = mp.mpf(0), mp.mpf(0)
                for j in range(w.n_theta):
                    for i in range(len(tab[key][j])):
                        b, W, K, Ct, C0 = tab[key][j][i]
                        ref = [si * b, s * W, si * K.real, si * K.imag, s * Ct.real, s * Ct.imag,
                               s * C0.real, s * C0.imag][c]
                        v = sum(mp.mpf(x) for x in got[which][c, j, i])
                        worst = max(worst, abs(v - ref))
                        # K can cancel to zero: scale its error by the cancelling terms
                        mx = max(mx, abs(ref), abs(si * b * Ct) if c in (2, 3) else 0)
                rel = worst / mx if mx else worst
                report.append((which, c, float(rel)))
        _note("  coefficient rel errors: %s" % report)
        for which, c, rel in report:
            assert rel <= TOL[words] / 100, (which, c, rel)


def test_batched_equals_single_bitwise():
    ws = [inputs.C1.with_(n_r=40 + 7 * k, n_theta=nth, rstar_min=60.0, rstar_max=150.0, m=k % 3,
                          a_over_M=0.2 * k, words=2, seed=k)
          for k, nth in enumerate((8, 16, 12, 32))]
    _note("batched vs single, %d instances" % len(ws))
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 2)
    b.set_tile(6)
    fields = [inputs.initial_fields(w) for w in ws]
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    b.step(15)
    for k, w in enumerate(ws):
        single = _run_gpu(w, fields[k], 15, tile=6)
        for f in range(4):
            assert np.array_equal(b.read_field(k, f), single[f]), (k, f)
    b.close()


# launch shapes: (sweep, segcols, block); the wide sweep with several theta
# groups per block, one group per block, segments of one node, ragged tails
SHAPES = [(T.SWEEP_SEGMENT, 8, 0), (T.SWEEP_SEGMENT, 3, 64), (T.SWEEP_WIDE, 8, 0), (T.SWEEP_WIDE, 1, 0),
          (T.SWEEP_WIDE, 5, 64), (T.SWEEP_WIDE, 13, 256), (T.SWEEP_WIDE, 40, 0), (T.SWEEP_WIDE2, 8, 0),
          (T.SWEEP_WIDE2, 1, 0), (T.SWEEP_WIDE2, 5, 64), (T.SWEEP_WIDE2, 11, 128), (T.SWEEP_WIDE2, 40, 512),
          (T.SWEEP_WIDE, 13, 128), (T.SWEEP_WIDE2, 3, 256)]


@pytest.mark.parametrize("words", [1, 2, 4])
def test_sweeps_and_launch_shapes_are_bitwise(words):
    """Every sweep and launch shape gives the same bits (they run the same
    per-point arithmetic in the same order), also when the segment length does
    not divide n_r and n_theta does not divide the block."""
    w = inputs.C1.with_(n_r=53, n_theta=24, rstar_min=60.0, rstar_max=150.0, words=words, m=1, a_over_M=0.7)
    fields = inputs.initial_fields(w)
    ref = None
    for sweep, seg, block in SHAPES:
        if (words == 4 and block > 256) or (sweep == T.SWEEP_WIDE2 and words != 1):
            continue
        _note("shape words=%d sweep=%d segcols=%d block=%d" % (words, sweep, seg, block))
        got = _run_gpu(w, fields, 9, tile=seg, sweep=sweep, block=block)
        if ref is None:
            ref = got
            assert rel_linf(got, oracle_run(w, fields, 9)) <= TOL[words]
        for f in range(4):
            assert np.array_equal(got[f], ref[f]), (sweep, seg, block, f)


@pytest.mark.parametrize("sweep", [T.SWEEP_WIDE, T.SWEEP_WIDE2], ids=["wide", "wide2"])
def test_fp64_coefficient_row_modes_are_bitwise(sweep, monkeypatch):
    """n_theta a multiple of 64: the FP64 wide sweeps read the radial rows with
    scalar loads; TEUK_NO_SCALAR_ROWS stages them in LDS instead.  Same bits,
    and both match the oracle."""
    w = inputs.C1.with_(n_r=45, n_theta=64, rstar_min=60.0, rstar_max=150.0, words=1, m=2, a_over_M=0.9)
    fields = inputs.initial_fields(w)
    _note("row modes sweep %d" % sweep)
    got = _run_gpu(w, fields, 8, tile=9, sweep=sweep, block=128)
    monkeypatch.setenv("TEUK_NO_SCALAR_ROWS", "1")
    lds_rows = _run_gpu(w, fields, 8, tile=9, sweep=sweep, block=128)
    for f in range(4):
        assert np.array_equal(got[f], lds_rows[f]), f
    assert rel_linf(got, oracle_run(w, fields, 8)) <= TOL[1]


@pytest.mark.parametrize("words", [1, 2, 4])
def test_largest_theta_grid(words):
    """n_theta = 256, the largest the library takes: the default sweep (wide where
    its slots fit in 64 KiB of LDS, else segment) against the oracle, and every
    sweep that accepts the grid gives the same bits."""
    w = inputs.C1.with_(n_r=13, n_theta=256, rstar_min=90.0, rstar_max=110.0, words=words, m=2, a_over_M=0.6)
    fields = inputs.initial_fields(w)
    _note("n_theta 256 words=%d" % words)
    got = _run_gpu(w, fields, 4, tile=5)
    assert rel_linf(got, oracle_run(w, fields, 4)) <= TOL[words]
    for sweep in ([T.SWEEP_SEGMENT, T.SWEEP_WIDE] + ([T.SWEEP_WIDE2] if words == 1 else [])):
        try:
            other = _run_gpu(w, fields, 4, tile=5, sweep=sweep)
        except T.TeukError as ex:           # wide slots beyond the device's LDS
            _note("  sweep %d not available: %s" % (sweep, ex))
            continue
        for f in range(4):
            assert np.array_equal(got[f], other[f]), (sweep, f)


# (words, n_theta, block, segcols, steps per launch): blocks at both radial
# boundaries, ragged last segments, step counts that leave a remainder
# (words, n_theta, block, segcols, steps per launch); the FP64 two-step cases
# with 64 and 128 theta rows take three or four unrolled iterations, the last
# one with a one-column last segment (the second-to-last block reaches the
# right boundary)
FUSED = [(1, 32, 256, 4, 4), (1, 32, 256, 9, 2), (1, 64, 512, 4, 4), (1, 64, 512, 10, 2),
         (1, 64, 256, 8, 2), (1, 64, 256, 12, 2), (1, 128, 512, 8, 2), (1, 64, 512, 23, 2),
         (2, 32, 256, 4, 4), (2, 32, 512, 12, 2), (2, 64, 512, 3, 4)]


@pytest.mark.parametrize("words,nth,block,seg,fuse", FUSED, ids=["w%d-t%d-b%d-s%d-f%d" % c for c in FUSED])
def test_fused_steps_are_bitwise(words, nth, block, seg, fuse):
    """Several steps per launch give the same bits as one step per launch, with
    and without graph replay, and match the oracle."""
    w = inputs.C1.with_(n_r=47, n_theta=nth, rstar_min=60.0, rstar_max=150.0, words=words, m=1, a_over_M=0.8)
    fields = inputs.initial_fields(w)
    _note("fused words=%d n_theta=%d block=%d segcols=%d fuse=%d" % (words, nth, block, seg, fuse))
    ref = _run_gpu(w, fields, 11, tile=seg, sweep=T.SWEEP_WIDE, block=block)
    for graph in (0, 4):
        h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), words)
        h.set_sweep(T.SWEEP_WIDE)
        h.set_launch(seg, block)
        h.set_fuse(fuse)
        h.use_graph(graph)
        h.set_initial(*fields)
        h.step(11)
        got = h.fields()
        assert h.steps_done == 11
        h.close()
        for f in range(4):
            assert np.array_equal(got[f], ref[f]), (graph, f)
    assert rel_linf(ref, oracle_run(w, fields, 11)) <= TOL[words]


# FP64 fused launches beyond the forms above: (sweep, n_theta, block, segcols,
# steps per launch) -- runs of two columns (up to three iterations) with two
# or four steps, runs of one with four steps and three or four iterations;
# the segment lengths leave ragged last segments, some shorter than the steps
FUSED_FP64 = [(T.SWEEP_WIDE2, 64, 256, 8, 2), (T.SWEEP_WIDE2, 128, 256, 8, 2), (T.SWEEP_WIDE2, 128, 256, 6, 2),
              (T.SWEEP_WIDE2, 64, 512, 12, 2), (T.SWEEP_WIDE2, 64, 256, 11, 2), (T.SWEEP_WIDE2, 64, 512, 16, 4),
              (T.SWEEP_WIDE2, 128, 512, 16, 4), (T.SWEEP_WIDE2, 64, 512, 13, 4), (T.SWEEP_WIDE, 64, 256, 8, 4),
              (T.SWEEP_WIDE, 128, 512, 8, 4), (T.SWEEP_WIDE, 64, 512, 23, 4)]


@pytest.mark.parametrize("sweep,nth,block,seg,fuse", FUSED_FP64,
                         ids=["r%d-t%d-b%d-s%d-f%d" % (c[0], c[1], c[2], c[3], c[4]) for c in FUSED_FP64])
def test_fused_fp64_forms_are_bitwise(sweep, nth, block, seg, fuse):
    """Several steps per launch give the bits of single steps (default
    launch), with and without graph replay."""
    w = inputs.C1.with_(n_r=47, n_theta=nth, rstar_min=60.0, rstar_max=150.0, m=1, a_over_M=0.8)
    fields = inputs.initial_fields(w)
    _note("fused FP64: sweep=%d n_theta=%d block=%d segcols=%d fuse=%d" % (sweep, nth, block, seg, fuse))
    ref = _run_gpu(w, fields, 11)
    for graph in (0, 4):
        h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 1)
        h.set_sweep(sweep)
        h.set_launch(seg, block)
        h.set_fuse(fuse)
        h.use_graph(graph)
        h.set_initial(*fields)
        h.step(11)
        got = h.fields()
        h.close()
        for f in range(4):
            assert np.array_equal(got[f], ref[f]), (graph, f)


def test_fused_batch_equals_single():
    ws = [inputs.C1.with_(n_r=30 + 11 * k, n_theta=32, rstar_min=60.0, rstar_max=150.0, m=k, a_over_M=0.3 * k,
                          words=2, seed=k) for k in range(3)]
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 2)
    b.set_sweep(T.SWEEP_WIDE)
    b.set_launch(4, 256)
    b.set_fuse(4)
    fields = [inputs.initial_fields(w) for w in ws]
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    b.step(9)
    for k, w in enumerate(ws):
        single = _run_gpu(w, fields[k], 9, tile=4, sweep=T.SWEEP_WIDE, block=256)
        for f in range(4):
            assert np.array_equal(b.read_field(k, f), single[f]), (k, f)
    b.close()


@pytest.mark.parametrize("words", [1, 2])
def test_autotuned_shape_is_bitwise(words, tmp_path, monkeypatch):
    """The autotuner (fused candidates included) leaves the handle on a shape
    that gives the same bits as the default launch."""
    import torch
    from paper_1006_0663_amd import autotune
    monkeypatch.setenv("TEUK_TUNE_CACHE", str(tmp_path / "cache.json"))
    w = inputs.C1.with_(n_r=47, n_theta=32, rstar_min=60.0, rstar_max=150.0, words=words, m=1, a_over_M=0.8)
    fields = inputs.initial_fields(w)
    ref = _run_gpu(w, fields, 11)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), words)
    h.set_stream(stream.cuda_stream)
    h.set_initial(*fields)
    best = autotune.tune(h, words, [(w.n_r, w.n_theta)], torch, stream, steps=8, reps=1)
    _note("autotuned words=%d: %s" % (words, best))
    assert len(best) == 5 and best[3] in (1, 2, 4)
    h.set_initial(*fields)
    h.step(11)
    got = h.fields()
    h.close()
    for f in range(4):
        assert np.array_equal(got[f], ref[f]), f


@pytest.mark.parametrize("n_r", [3, 4, 5, 9])
def test_fused_tiny_radial_grids(n_r):
    """Fused launches on grids with fewer r* nodes than a segment (one work
    item that touches both radial boundaries) match single steps bitwise."""
    w = inputs.C1.with_(n_r=n_r, n_theta=64, rstar_min=95.0, rstar_max=95.0 + 3.0 * n_r, m=2, a_over_M=0.5)
    fields = inputs.initial_fields(w)
    ref = _run_gpu(w, fields, 9)
    for sweep, seg, block, fuse in ((T.SWEEP_WIDE, 4, 256, 2), (T.SWEEP_WIDE, 4, 256, 4),
                                    (T.SWEEP_WIDE2, 16, 512, 4), (T.SWEEP_WIDE2, 8, 256, 2)):
        _note("fused tiny grid: n_r=%d sweep=%d segcols=%d block=%d fuse=%d" % (n_r, sweep, seg, block, fuse))
        h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 1)
        h.set_sweep(sweep)
        h.set_launch(seg, block)
        h.set_fuse(fuse)
        h.set_initial(*fields)
        h.step(9)
        got = h.fields()
        h.close()
        for f in range(4):
            assert np.array_equal(got[f], ref[f]), (sweep, seg, block, fuse, f)


def test_fused_fp64_batch_equals_single():
    """An FP64 batch of uneven instances with four steps per launch and runs of
    two columns gives each instance the bits of its own single-step run."""
    ws = [inputs.C1.with_(n_r=30 + 13 * k, n_theta=(64, 128, 64)[k], rstar_min=60.0, rstar_max=150.0, m=k,
                          a_over_M=0.3 * k, seed=k) for k in range(3)]
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 1)
    b.set_sweep(T.SWEEP_WIDE2)
    b.set_launch(8, 512)
    b.set_fuse(4)
    fields = [inputs.initial_fields(w) for w in ws]
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    b.use_graph(8)
    b.step(13)
    for k, w in enumerate(ws):
        single = _run_gpu(w, fields[k], 13)
        for f in range(4):
            assert np.array_equal(b.read_field(k, f), single[f]), (k, f)
    b.close()


def test_fuse_rejects_unsupported_shapes():
    w = inputs.C1.with_(n_r=40, n_theta=32, words=4)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 4)
    with pytest.raises(T.TeukError):
        h.set_fuse(2)                       # quad-double has no fused form
    with pytest.raises(T.TeukError):
        h.set_fuse(3)
    h.close()
    w = inputs.C1.with_(n_r=40, n_theta=32, words=1)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 1)
    h.set_sweep(T.SWEEP_WIDE)
    h.set_launch(40, 256)
    with pytest.raises(T.TeukError):
        h.set_fuse(4)                       # 40 + 12 columns need more than two iterations
    h.set_launch(4, 256)
    h.set_fuse(4)                           # the previous failure left the handle usable
    h.close()


def test_wide2_rejected_for_multiword():
    w = inputs.C1.with_(n_r=20, n_theta=8, words=2)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 2)
    with pytest.raises(T.TeukError) as ex:
        h.set_sweep(T.SWEEP_WIDE2)
    assert ex.value.code == T.TEUK_ENOTSUP
    assert h.sweep == T.SWEEP_WIDE
    h.close()


@pytest.mark.parametrize("sweep", [T.SWEEP_WIDE, T.SWEEP_WIDE2], ids=["wide", "wide2"])
def test_wide_sweep_batch_equals_single(sweep):
    ws = [inputs.C1.with_(n_r=40 + 9 * k, n_theta=nth, rstar_min=60.0, rstar_max=150.0, m=k % 3,
                          a_over_M=0.25 * k, words=1, seed=k)
          for k, nth in enumerate((8, 40, 16, 64))]
    _note("wide batched vs single, %d instances, sweep %d" % (len(ws), sweep))
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w)) for w in ws], 1)
    b.set_sweep(sweep)
    b.set_launch(7, 0)
    fields = [inputs.initial_fields(w) for w in ws]
    for k, f in enumerate(fields):
        b.set_initial(k, *f)
    b.step(11)
    for k, w in enumerate(ws):
        single = _run_gpu(w, fields[k], 11, tile=7, sweep=sweep)
        for f in range(4):
            assert np.array_equal(b.read_field(k, f), single[f]), (k, f)
    b.close()


def test_checkpoint_restart_and_graph_are_bitwise():
    w = inputs.C1.with_(n_r=50, n_theta=16, rstar_min=60.0, rstar_max=150.0, words=4)
    fields = inputs.initial_fields(w)
    _note("checkpoint/graph qd 50x16")
    full = _run_gpu(w, fields, 10)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 4)
    h.set_initial(*fields)
    h.step(5)
    mid = h.fields()
    assert h.steps_done == 5
    h.set_initial(*mid)
    h.set_step_index(5)
    h.step(5)
    assert h.steps_done == 10
    for f in range(4):
        assert np.array_equal(h.read_field(f), full[f])
    h.set_initial(*fields)
    h.use_graph(4)
    h.step(10)                    # 2 graph replays + 2 plain launches
    for f in range(4):
        assert np.array_equal(h.read_field(f), full[f])
    h.set_initial(*fields)
    h.use_graph(3)                # an odd launch count: replays alternate between the two graphs
    before = h.graph_replays      # (counted since the handle was created)
    h.step(10)
    assert h.graph_replays - before == 3
    for f in range(4):
        assert np.array_equal(h.read_field(f), full[f])
    h.set_initial(*fields)
    h.prepare_graph()             # both graphs captured up front; results unchanged
    h.step(10)
    for f in range(4):
        assert np.array_equal(h.read_field(f), full[f])
    h.close()


def test_round_trip_and_edges():
    # smallest legal grid, zero steps, boundary columns forced to zero
    w = inputs.C1.with_(n_r=3, n_theta=5, rstar_min=0.0, rstar_max=10.0, words=2)
    rng = np.random.default_rng(0)
    f = [rng.standard_normal((5, 3, 2)) for _ in range(4)]
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 2)
    h.set_initial(*f)
    h.step(0)
    for c in range(4):
        got = h.read_field(c)
        assert np.all(got[:, [0, 2]] == 0)
        # interior values are renormalised exactly: same sum, |lo| <= ulp(hi)/2
        assert np.array_equal(got[:, 1, 0] + got[:, 1, 1], f[c][:, 1, 0] + f[c][:, 1, 1])
        assert np.all(got[:, 1, 0] == (f[c][:, 1, 0] + f[c][:, 1, 1]))
    h.step(3)
    ref = oracle_run(w, [h_ for h_ in [np.where(np.arange(3)[None, :, None] % 2 == 1, x, 0) for x in f]], 3)
    got = h.fields()
    assert rel_linf(got, ref) <= TOL[2]
    assert h.check_finite()
    h.close()


@pytest.mark.parametrize("words", [1, 2, 4])
def test_device_arithmetic_matches_host(words):
    rng = np.random.default_rng(words)
    a = rng.standard_normal((257, words)) * np.array([1, 2 ** -60, 2 ** -120, 2 ** -180][:words])
    b = rng.standard_normal((257, words)) * np.array([1, 2 ** -60, 2 ** -120, 2 ** -180][:words])
    for op in (0, 1, 2, 3, 4):
        assert np.array_equal(T.arith(words, op, a, b, device=True), T.arith(words, op, a, b)), op


def _mp_words(x, W):
    """Nearest W-word non-overlapping float64 expansion of an mp number."""
    out = []
    for _ in range(W):
        v = float(x)
        out.append(v)
        x = x - mp.mpf(v)
    return out


def _oracle_planes(w, tab):
    """The eight scaled coefficient planes of teuk_set_coefficients (half
    nodes, nodes), rounded to the workload's words from the oracle's tables."""
    W = w.words
    out = {}
    with mp.workprec(450):
        scal = {0: (tab["dt"] / 2, tab["dt"] / 2 / tab["h"]), 1: (tab["dt"], tab["dt"] / tab["h"])}
        for which, key in ((0, "half"), (1, "full")):
            s_, si = scal[which]
            nr = len(tab[key][0])
            a = np.empty((8, w.n_theta, nr, W))
            for j in range(w.n_theta):
                for i in range(nr):
                    b, Wc, K, Ct, C0 = tab[key][j][i]
                    vals = [si * b, s_ * Wc, si * K.real, si * K.imag, s_ * Ct.real, s_ * Ct.imag,
                            s_ * C0.real, s_ * C0.imag]
                    for c in range(8):
                        a[c, j, i] = _mp_words(vals[c], W)
            out[which] = a
    return out


@pytest.mark.parametrize("words,fuse", [(1, 4), (1, 1), (2, 1), (2, 2)])
def test_stepping_on_injected_oracle_coefficients(words, fuse):
    """The oracle's 450-bit coefficients, rounded to the working words and
    injected through teuk_set_coefficients, drive the step (for FP64 this is
    the stored-plane kernel, a separate instantiation from the per-point one),
    and the result matches the oracle run on its own coefficients.  A handle
    set to fused launches first: the switch to stored planes falls back to one
    step per launch and the next step(1) runs (and is right)."""
    w = inputs.C1.with_(n_r=47, n_theta=64, rstar_min=60.0, rstar_max=150.0, words=words, m=1, a_over_M=0.8)
    fields = inputs.initial_fields(w)
    _note("injected oracle coefficients words=%d fuse=%d" % (words, fuse))
    tab = problem.build_tables(to_problem(w))
    planes = _oracle_planes(w, tab)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), words)
    h.set_sweep(T.SWEEP_WIDE2 if words == 1 else T.SWEEP_WIDE)
    h.set_launch(16 if words == 1 else 4, 512)
    h.set_fuse(fuse)
    h.set_coefficients(0, planes[0])
    h.set_coefficients(1, planes[1])
    for which in (0, 1):
        assert np.array_equal(h.coefficients(which), planes[which]), which
    h.set_initial(*fields)
    h.step(1)
    h.step(10)
    got = h.fields()
    h.close()
    err = rel_linf(got, oracle_run(w, fields, 11, tables=tab))
    _note("  rel Linf = %.3e" % err)
    assert err <= TOL[words]


def test_nonfinite_initial_data_is_refused():
    w = inputs.C1.with_(n_r=20, n_theta=8, rstar_min=60.0, rstar_max=150.0, words=2)
    fields = [np.array(f) for f in inputs.initial_fields(w)]
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), 2)
    h.set_initial(*fields)
    h.step(2)
    before = h.fields()
    for bad in (np.nan, np.inf, -np.inf):
        f = [x.copy() for x in fields]
        f[3][4, 7, 1] = bad
        with pytest.raises(T.TeukError) as ex:
            h.set_initial(*f)
        assert ex.value.code == T.TEUK_ENONFINITE
    after = h.fields()                       # nothing was uploaded
    for c in range(4):
        assert np.array_equal(before[c], after[c])
    f = [x.copy() for x in fields]
    f[0][3, 0, 0] = np.nan                   # a radial boundary node is set to zero, not checked
    h.set_initial(*f)
    assert h.check_finite()
    h.close()


@pytest.mark.parametrize("words", [1, 2])
def test_host_round_trip_is_bitwise(words):
    """The host round-trip measurement mode (state to host memory and back
    after every step) gives the same bits as resident stepping."""
    w = inputs.C1.with_(n_r=47, n_theta=32, rstar_min=60.0, rstar_max=150.0, words=words, m=2, a_over_M=0.6)
    fields = inputs.initial_fields(w)
    ref = _run_gpu(w, fields, 7)
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), words)
    h.use_graph(4)
    h.set_host_round_trip(True)
    h.set_initial(*fields)
    h.step(7)
    assert h.graph_replays == 0
    got = h.fields()
    h.set_host_round_trip(False)
    h.set_initial(*fields)
    h.step(7)
    again = h.fields()
    h.close()
    for c in range(4):
        assert np.array_equal(got[c], ref[c]), c
        assert np.array_equal(again[c], ref[c]), c
