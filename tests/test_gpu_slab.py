"""GPU checks of the persistent slab sweep (TEUK_SWEEP_SLAB): one launch per
call, each block keeping its r* segment resident and trading only the edge
values with its neighbours through global memory and flags.  It must give
the same bits as the wide sweep (which the parity tests pin to the oracle)
on every grid shape it accepts, match the oracle directly, keep the observer
series and the host round trip unchanged, turn an abandoned neighbour wait
into TEUK_EDEVICE, and refuse what it does not support."""
import sys

import numpy as np
import pytest

from paper_1006_0663_amd import inputs, teuk as T
from parity_util import oracle_run, rel_linf

pytestmark = pytest.mark.gpu

def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _grid(w):
    return T.make_grid(w.n_r, w.n_theta, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order)


def _handle(w, fields, sweep=None, segcols=None, block=0, fuse=1):
    h = T.Teuk(w.s, w.m, w.a_over_M, _grid(w), w.words)
    h.set_initial(*fields)
    if sweep is not None:
        h.set_sweep(sweep)
        if segcols:
            h.set_launch(segcols, block)
        h.set_fuse(fuse)
    return h


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


C2 = inputs.C2
# (label, workload, segcols, block, step calls): the headline grid in its
# benchmarked shape (256 segments of 16 nodes, one per compute unit); ragged
# last segments; a single segment (no neighbour exchange); n_theta 64 and
# 256; other spin weights and negative m.
CASES = [
    ("headline-16x512", C2, 16, 512, [100, 3]),
    ("headline-16x1024", C2, 16, 1024, [20, 20, 7]),
    ("ragged-1000x64", C2.with_(n_r=1000, n_theta=64), 16, 512, [37, 64, 1]),
    ("r1-200x64", C2.with_(n_r=200, n_theta=64), 4, 256, [50]),
    ("one-segment-16x64", C2.with_(n_r=16, n_theta=64), 16, 256, [20]),
    ("nth256-600x256", C2.with_(n_r=600, n_theta=256), 4, 1024, [9, 12]),
    ("s1-m-2-333x64", C2.with_(n_r=333, n_theta=64, s=1, m=-2, a_over_M=0.95), 8, 256, [7, 30]),
    ("s0-m0-a0-257x128", C2.with_(n_r=257, n_theta=128, s=0, m=0, a_over_M=0.0), 8, 512, [41]),
    # double-double (coefficients held in registers, one or two columns per lane)
    ("dd-1024x64", inputs.C3_PARITY, 4, 256, [13, 20]),
    ("dd-ragged-333x64-s1-m-2", inputs.C3_PARITY.with_(n_r=333, s=1, m=-2, a_over_M=0.95), 8, 256, [7, 30]),
    ("dd-300x128", C2.with_(n_r=300, words=2), 4, 512, [11]),
    ("dd-one-segment-8x64", inputs.C3_PARITY.with_(n_r=8), 8, 256, [9]),
    # quad-double (coefficients loaded per stage, one column per lane)
    ("qd-2048x64", inputs.C4, 8, 512, [3, 2]),
    ("qd-ragged-203x64-s-1-m2", inputs.C4.with_(n_r=203, s=-1, m=2, a_over_M=0.6), 4, 256, [4]),
]


@pytest.mark.parametrize("label,w,seg,block,calls", CASES, ids=[c[0] for c in CASES])
def test_slab_equals_wide_sweep_bitwise(label, w, seg, block, calls):
    fields = inputs.initial_fields(w)
    _note("slab %s: %dx%d segcols %d block %d calls %s" % (label, w.n_r, w.n_theta, seg, block, calls))
    ref = _handle(w, fields)
    h = _handle(w, fields, T.SWEEP_SLAB, seg, block)
    assert h.sweep == T.SWEEP_SLAB
    for n in calls:
        ref.step(n)
        h.step(n)
    got, want = h.fields(), ref.fields()
    assert h.steps_done == sum(calls)
    h.close()
    ref.close()
    assert _same(got, want)


ORACLE_CASES = [
    ("fp64-m2-61x64", inputs.C1.with_(n_r=61, n_theta=64, rstar_min=60.0, rstar_max=150.0, words=1), 4, 256),
    ("fp64-s2-m-2-45x64", inputs.C1.with_(n_r=45, n_theta=64, rstar_min=70.0, rstar_max=140.0, s=2, m=-2,
                                          a_over_M=0.9, words=1), 8, 256),
    ("dd-m3-a0.99-45x64", inputs.C4.with_(n_r=45, n_theta=64, rstar_min=60.0, rstar_max=150.0, m=3, words=2),
     4, 256),
    ("qd-m2-a0.99-37x64", inputs.C4.with_(n_r=37, n_theta=64, rstar_min=60.0, rstar_max=150.0, words=4), 8, 512),
]
TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60}


@pytest.mark.parametrize("label,w,seg,block", ORACLE_CASES, ids=[c[0] for c in ORACLE_CASES])
def test_slab_matches_oracle(label, w, seg, block):
    """Several segments with a ragged last one, against the oracle."""
    nsteps = 24
    fields = inputs.initial_fields(w)
    _note("slab oracle %s: %dx%d segcols %d steps %d" % (label, w.n_r, w.n_theta, seg, nsteps))
    h = _handle(w, fields, T.SWEEP_SLAB, seg, block)
    h.step(nsteps)
    got = h.fields()
    h.close()
    err = rel_linf(got, oracle_run(w, fields, nsteps, processes=8))
    _note("  rel Linf = %.3e" % err)
    assert err <= TOL[w.words]


def test_slab_cooperative_launch_is_bitwise(monkeypatch):
    """TEUK_SLAB_COOPERATIVE (read when the handle is created) launches the
    same kernel cooperatively: same bits."""
    w = C2.with_(n_r=700, n_theta=128)
    fields = inputs.initial_fields(w)
    a = _handle(w, fields, T.SWEEP_SLAB, 16, 1024)
    monkeypatch.setenv("TEUK_SLAB_COOPERATIVE", "1")
    b = _handle(w, fields, T.SWEEP_SLAB, 16, 1024)
    monkeypatch.delenv("TEUK_SLAB_COOPERATIVE")
    a.step(33)
    b.step(33)
    assert _same(a.fields(), b.fields())
    a.close()
    b.close()


def test_slab_observer_series_equals_wide_sweep():
    """Launches are cut where a record falls due: the series is the wide
    sweep's, record for record."""
    w = C2.with_(n_r=512, n_theta=128)
    fields = inputs.initial_fields(w)
    pts = [(100, 3), (256, 64), (400, 127)]
    out = []
    for sweep in (None, T.SWEEP_SLAB):
        h = _handle(w, fields, sweep, 16 if sweep else None, 512 if sweep else 0)
        h.set_observer(pts, every=7, capacity=64)
        h.step(30)
        h.step(23)
        out.append(h.read_observer())
        h.close()
    (sa, pa, na), (sb, pb, nb) = out
    assert na == nb == 53 // 7
    assert np.array_equal(sa, sb) and np.array_equal(pa, pb)


def test_slab_host_round_trip_is_bitwise():
    w = C2.with_(n_r=256, n_theta=64)
    fields = inputs.initial_fields(w)
    a = _handle(w, fields, T.SWEEP_SLAB, 8, 256)
    a.step(12)
    b = _handle(w, fields, T.SWEEP_SLAB, 8, 256)
    b.set_host_round_trip(True)
    b.step(12)
    assert _same(a.fields(), b.fields())
    a.close()
    b.close()


def test_slab_abandoned_wait_is_a_device_error(monkeypatch):
    """TEUK_FAULT=slab-abort sets the error word from the host before each
    launch, so the first wait that finds its flag missing gives up at once:
    the kernel ends early, the next synchronising call reports TEUK_EDEVICE
    and the handle stays failed; a new handle runs normally afterwards."""
    w = C2.with_(n_r=512, n_theta=64)
    fields = inputs.initial_fields(w)
    monkeypatch.setenv("TEUK_FAULT", "slab-abort")
    h = _handle(w, fields, T.SWEEP_SLAB, 8, 256)
    monkeypatch.delenv("TEUK_FAULT")
    h.set_observer([(100, 5)], every=3, capacity=8)
    h.step(10)                                  # launches; the error shows at the next sync
    with pytest.raises(T.TeukError) as ex:
        h.read_observer()                       # its records are not valid either
    assert ex.value.code == T.TEUK_EDEVICE and "neighbouring block" in str(ex.value)
    with pytest.raises(T.TeukError) as ex:
        h.fields()
    assert ex.value.code == T.TEUK_EDEVICE
    with pytest.raises(T.TeukError):
        h.step(1)                               # failed state is sticky
    h.close()
    ref = _handle(w, fields)
    g = _handle(w, fields, T.SWEEP_SLAB, 8, 256)
    ref.step(10)
    g.step(10)
    assert _same(g.fields(), ref.fields())
    ref.close()
    g.close()


def test_slab_refusals_and_fallbacks():
    w = C2.with_(n_r=300, n_theta=64)
    fields = inputs.initial_fields(w)
    h = _handle(w, fields)
    h.set_sweep(T.SWEEP_SLAB)                  # default block 256, shortest segments that fit
    assert h.sweep == T.SWEEP_SLAB
    with pytest.raises(T.TeukError) as ex:
        h.set_launch(6, 256)                    # 6 is not 1, 2 or 4 times 256 / 64
    assert ex.value.code == T.TEUK_EINVAL
    with pytest.raises(T.TeukError) as ex:
        h.set_fuse(2)
    assert ex.value.code == T.TEUK_EINVAL
    assert h.sweep == T.SWEEP_SLAB              # refused requests leave the plan as it was
    h.step(5)
    # injected coefficients exist only as planes: the handle falls back to the default sweep
    h.set_coefficients(1, h.coefficients(1))
    assert h.sweep != T.SWEEP_SLAB
    h.step(5)
    h.close()
    # n_theta not 64, 128 or 256, double-double with four columns per lane, batches
    with pytest.raises(T.TeukError) as ex:
        g = _handle(w.with_(words=2), inputs.initial_fields(w.with_(words=2)))
        try:
            g.set_sweep(T.SWEEP_SLAB)
            g.set_launch(16, 256)
        finally:
            g.close()
    assert ex.value.code == T.TEUK_EINVAL
    for ww, code in ((w.with_(n_theta=32), T.TEUK_ENOTSUP), (w.with_(n_theta=192), T.TEUK_ENOTSUP)):
        g = _handle(ww, inputs.initial_fields(ww))
        with pytest.raises(T.TeukError) as ex:
            g.set_sweep(T.SWEEP_SLAB)
        assert ex.value.code == code
        g.close()
    b = T.TeukBatch([(w.s, w.m, w.a_over_M, _grid(w))] * 2, 1)
    with pytest.raises(T.TeukError) as ex:
        b.set_sweep(T.SWEEP_SLAB)
    assert ex.value.code == T.TEUK_ENOTSUP
    b.close()
