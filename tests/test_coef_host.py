"""The library's coefficient-pass routines, run on the host through a test
fixture (tests/host_emul), against the oracle's 450-bit Kerr factors."""
import ctypes
import os

import mpmath as mp
import numpy as np
import pytest

from paper_1006_0663_amd import inputs
from oracle import problem
from parity_util import to_problem

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "host_emul", "libcoefhost.so")
TOL = {1: 1e-14, 2: 1e-30, 4: 1e-62}


def host_coefficients(w, dd_rows=False):
    """The planes of the coefficient pass (dd_rows: of the double-double
    per-point mode, built from double-double radial rows)."""
    L = ctypes.CDLL(LIB)
    D = ctypes.POINTER(ctypes.c_double)
    L.coef_host.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] + [ctypes.c_int] * 2 + [ctypes.c_double] * 4 + \
        [ctypes.c_int, D, D, D, D]
    L.coef_host_dd_rows.argtypes = L.coef_host.argtypes[1:]
    W, nr, nth, R = w.words, w.n_r, w.n_theta, w.angular_order // 2
    ch = np.zeros((8, W, nr - 1, nth))
    cf = np.zeros((8, W, nr, nth))
    wt = np.zeros((2 * R + 1, W, nth))
    scal = np.zeros(8)
    p = lambda a: a.ctypes.data_as(D)
    args = (w.s, w.m, w.a_over_M, nr, nth, w.rstar_min, w.rstar_max, w.cfl, w.mass, w.angular_order,
            p(ch), p(cf), p(wt), p(scal))
    if dd_rows:
        assert W == 2
        L.coef_host_dd_rows(*args)
    else:
        L.coef_host(W, *args)
    return ch, cf, wt, scal


def _val(words):
    return sum((mp.mpf(float(x)) for x in words), mp.mpf(0))


@pytest.mark.parametrize("words,dd_rows", [(1, False), (2, False), (4, False), (2, True)],
                         ids=["fp64", "dd", "qd", "dd-per-point"])
@pytest.mark.parametrize("a,m", [(0.9, 3), (0.0, 2), (0.99, -1)])
def test_host_coefficients_match_oracle(words, dd_rows, a, m):
    w = inputs.C2.with_(n_r=17, n_theta=8, words=words, a_over_M=a, m=m)
    ch, cf, wt, scal = host_coefficients(w, dd_rows)
    tab = problem.build_tables(to_problem(w))
    with mp.workprec(450):
        assert abs(_val(scal[4:4 + words]) - tab["dt"]) <= TOL[words] * tab["dt"]
        scales = {0: (tab["dt"] / 2, tab["dt"] / 2 / tab["h"]), 1: (tab["dt"], tab["dt"] / tab["h"])}
        bad = []
        for which, key, arr in ((0, "half", ch), (1, "full", cf)):
            s, si = scales[which]
            for c in range(8):
                worst, mx = mp.mpf(0), mp.mpf(0)
                for j in range(w.n_theta):
                    for i in range(len(tab[key][j])):
                        b, W, K, Ct, C0 = tab[key][j][i]
                        ref = [si * b, s * W, si * K.real, si * K.imag, s * Ct.real, s * Ct.imag,
                               s * C0.real, s * C0.imag][c]
                        worst = max(worst, abs(_val(arr[c, :, i, j]) - ref))
                        # K = b d_r*b - b Ct - Cs can cancel to zero (s = -2, a = 0):
                        # measure its error against the size of the cancelling terms
                        mx = max(mx, abs(ref), abs(si * b * Ct) if c in (2, 3) else 0)
                rel = worst / mx if mx else worst
                if rel > TOL[words]:
                    bad.append((key, c, float(rel)))
        # angular weights: d2_k + cot d1_k (ghost sign), V on the centre tap
        R = tab["reach"]
        for j in range(w.n_theta):
            for k in range(-R, R + 1):
                ref = tab["d2"][k + R] + tab["cot"][j] * tab["d1"][k + R]
                if (j + k < 0 or j + k >= w.n_theta) and tab["parity"] < 0:
                    ref = -ref
                if k == 0:
                    ref += tab["V"][j]
                if abs(_val(wt[k + R, :, j]) - ref) > TOL[words] * 10 * (1 + abs(ref)):
                    bad.append(("wt", j, k, float(abs(_val(wt[k + R, :, j]) - ref))))
        assert not bad, bad
