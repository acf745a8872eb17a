"""CPU checks of the library: it loads, exports every declared symbol, validates
arguments on the host, and its multiword arithmetic meets the published error
bounds (host build of the same routines the kernels use)."""
import os
import random
import re

import mpmath as mp
import numpy as np
import pytest

from paper_1006_0663_amd import teuk as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "teuk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(teuk_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) > 25
    L = T.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(T._SIGS), set(names) ^ set(T._SIGS)


def test_validation_without_gpu():
    L = T.lib()
    ok = T.make_grid(256, 32, -50, 250)
    assert L.teuk_validate(-2, 2, 0.5, ok, 2) == T.TEUK_OK
    bad = [(-3, 2, 0.5, ok, 2), (-2, 2, 1.0, ok, 2), (-2, 2, 0.5, ok, 3),
           (-2, 2, 0.5, T.make_grid(256, 4, -50, 250), 2), (-2, 2, 0.5, T.make_grid(2, 32, -50, 250), 2),
           (-2, 2, 0.5, T.make_grid(256, 32, 50, 50), 2), (-2, 2, 0.5, T.make_grid(256, 32, -50, 250, cfl=0), 2),
           (0, 0, 0.1, T.make_grid(64, 16, 2, 10, mass=0.0), 1), (0, 0, 0.0, T.make_grid(64, 16, -2, 10, mass=0.0), 1),
           (-2, 2, 0.5, T.make_grid(256, 32, -50, 250, angular_order=4), 2)]
    for args in bad:
        assert L.teuk_validate(*args) == T.TEUK_EINVAL, args
        assert L.teuk_last_error()
    assert L.teuk_validate(0, 0, 0.0, T.make_grid(64, 16, 2, 10, mass=0.0), 1) == T.TEUK_OK
    assert L.teuk_validate(-2, 2, 0.5, T.make_grid(256, 512, -50, 250), 2) == T.TEUK_ENOTSUP


def test_create_rejects_before_touching_a_device():
    with pytest.raises(T.TeukError) as e:
        T.Teuk(-2, 2, 1.5, T.make_grid(256, 32, -50, 250), 2)
    assert e.value.code == T.TEUK_EINVAL


def _words(x, n):
    out = []
    for _ in range(n):
        w = float(x)
        out.append(w)
        x -= mp.mpf(w)
    return out


def _val(ws):
    return sum((mp.mpf(w) for w in ws), mp.mpf(0))


def _rand(rng, W, lo, hi, signed=True):
    x = mp.mpf(rng.uniform(lo, hi)) * (1 + mp.mpf(rng.random()) * mp.mpf(2) ** -60
                                         + mp.mpf(rng.random()) * mp.mpf(2) ** -130)
    if signed and rng.random() < 0.5:
        x = -x
    return x


@pytest.mark.parametrize("W,bound_add,bound_mul", [(1, 2 ** -53, 2 ** -53), (2, 3 * 2 ** -106, 4 * 2 ** -106),
                                                   (4, 2 ** -205, 2 ** -205)])
def test_host_arithmetic_error_bounds(W, bound_add, bound_mul):
    """add/sub: |err| <= bound (|a| + |b|); mul: relative; div, sqrt: relative (two-ulp-ish)."""
    rng = random.Random(5 + W)
    with mp.workprec(500):
        xs = [_rand(rng, W, 0.01, 10) for _ in range(300)]
        ys = [_rand(rng, W, 0.01, 10) for _ in range(300)]
        # near-cancellation pairs
        ys[:60] = [-x * (1 + mp.mpf(2) ** -(rng.randint(1, 150))) for x in xs[:60]]
        A = np.array([_words(x, W) for x in xs])
        B = np.array([_words(y, W) for y in ys])
        Ax, Bx = [_val(r) for r in A], [_val(r) for r in B]
        for op, f, kind, bound in ((0, lambda a, b: a + b, "abs", bound_add), (1, lambda a, b: a - b, "abs", bound_add),
                                   (2, lambda a, b: a * b, "rel", bound_mul), (4, lambda a, b: a / b, "rel", 4 * bound_mul)):
            O = T.arith(W, op, A, B)
            for k in range(len(xs)):
                exact = f(Ax[k], Bx[k])
                err = abs(_val(O[k]) - exact)
                scale = (abs(Ax[k]) + abs(Bx[k])) if kind == "abs" else abs(exact)
                assert err <= bound * scale, (op, k, float(mp.log(err / scale, 2)))
        Aabs = A * np.sign(A[:, :1])             # negate whole expansions, not words
        O = T.arith(W, 5, Aabs, B)
        for k in range(len(xs)):
            exact = mp.sqrt(abs(Ax[k]))
            assert abs(_val(O[k]) - exact) <= 2 * bound_mul * exact


@pytest.mark.parametrize("W,bound", [(1, 2 ** -50), (2, 2 ** -102), (4, 2 ** -204)])
def test_host_transcendentals(W, bound):
    rng = random.Random(9)
    with mp.workprec(500):
        xs = [_rand(rng, W, 0.05, 1.5) for _ in range(40)]
        A = np.array([_words(x, W) for x in xs])
        Ax = [_val(r) for r in A]
        for op, f in ((6, mp.exp), (8, mp.sin), (9, mp.cos)):
            O = T.arith(W, op, A, A)
            for k in range(len(xs)):
                assert abs(_val(O[k]) - f(Ax[k])) <= bound, (op, k)
        P = A * np.sign(A[:, :1]) * 7
        Px = [_val(r) for r in P]
        O = T.arith(W, 7, P, P)
        for k in range(len(xs)):
            assert abs(_val(O[k]) - mp.log(Px[k])) <= bound * max(1, abs(mp.log(Px[k]))), k


def test_injected_allocation_failure_is_reported(monkeypatch):
    """TEUK_FAULT=alloc makes creation fail with TEUK_ENOMEM after validation
    and before any device call, so the error path is testable without a GPU."""
    monkeypatch.setenv("TEUK_FAULT", "alloc")
    for create in (lambda: T.Teuk(-2, 2, 0.5, T.make_grid(64, 16, -50, 250), 2),
                   lambda: T.TeukBatch([(-2, 2, 0.5, T.make_grid(64, 16, -50, 250))], 4)):
        with pytest.raises(T.TeukError) as e:
            create()
        assert e.value.code == T.TEUK_ENOMEM
        assert "TEUK_FAULT" in T.lib().teuk_last_error().decode()


def test_null_arguments_are_rejected():
    L = T.lib()
    assert L.teuk_step(None, 1) == T.TEUK_EINVAL
    assert L.teuk_read_field(None, 0, None) == T.TEUK_EINVAL
    assert L.teuk_set_launch(None, 4, 0) == T.TEUK_EINVAL
    assert L.teuk_set_sweep(None, 1) == T.TEUK_EINVAL
    assert L.teuk_batch_set_sweep(None, 1) == T.TEUK_EINVAL
    assert L.teuk_get_sweep(None) == T.TEUK_EINVAL
    assert L.teuk_set_fuse(None, 2) == T.TEUK_EINVAL
    assert L.teuk_batch_set_fuse(None, 2) == T.TEUK_EINVAL
    assert L.teuk_destroy(None) == T.TEUK_OK
    assert L.teuk_arith_host(3, 0, None, None, None, 1) == T.TEUK_EINVAL


@pytest.mark.parametrize("words", [1, 2, 4])
def test_grid_size_limit_of_32_bit_plane_offsets(words):
    """The step kernels address one word plane of the eight coefficient
    components with 32-bit offsets: validation takes 8 * words * n_r * n_theta
    up to 2^32 - 1 doubles and answers TEUK_ENOTSUP from 2^32 on, in every
    precision, for FP64 too (its stored-plane mode after
    teuk_set_coefficients uses the same offsets)."""
    L = T.lib()
    nth = 256
    limit_points = (1 << 32) // (8 * words)          # first rejected point count
    n_r_bad = limit_points // nth
    assert n_r_bad * nth * 8 * words == 1 << 32
    assert L.teuk_validate(-2, 2, 0.5, T.make_grid(n_r_bad, nth, -50, 250), words) == T.TEUK_ENOTSUP
    assert "2^32" in L.teuk_last_error().decode()
    assert L.teuk_validate(-2, 2, 0.5, T.make_grid(n_r_bad - 1, nth, -50, 250), words) == T.TEUK_OK
    # a point count just below the limit that no n_theta of 256 reaches
    assert L.teuk_validate(-2, 2, 0.5, T.make_grid(limit_points // 255 - 1, 255, -50, 250), words) == T.TEUK_OK
    assert L.teuk_validate(-2, 2, 0.5, T.make_grid(limit_points // 200 + 1, 200, -50, 250), words) == T.TEUK_ENOTSUP


def test_new_entry_points_reject_null_handles():
    L = T.lib()
    assert L.teuk_prepare_graph(None) == T.TEUK_EINVAL
    assert L.teuk_batch_prepare_graph(None) == T.TEUK_EINVAL
    assert L.teuk_graph_replays(None) == -1
    assert L.teuk_set_host_round_trip(None, 1) == T.TEUK_EINVAL
    assert L.teuk_set_observer(None, 0, None, None, 1, 1) == T.TEUK_EINVAL
    assert L.teuk_read_observer(None, 0, None, None, None) == T.TEUK_EINVAL
