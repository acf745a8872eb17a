"""The step kernel's own stage arithmetic (lw_stage, averages, differences,
folded angular weights), run on the host by the test fixture in
tests/host_emul, against the oracle: pins the stepping code without a GPU."""
import ctypes

import numpy as np
import pytest

from paper_1006_0663_amd import inputs
from parity_util import oracle_run, rel_linf
from test_coef_host import LIB, host_coefficients

TOL = {1: 1e-12, 2: 1e-28, 4: 1e-60}


def host_steps(w, fields, nsteps):
    D = ctypes.POINTER(ctypes.c_double)
    L = ctypes.CDLL(LIB)
    L.step_host.argtypes = [ctypes.c_int] * 4 + [D] * 4 + [D, ctypes.c_int]
    ch, cf, wt, scal = host_coefficients(w)
    u = np.zeros((4, w.words, w.n_r, w.n_theta))
    for c in range(4):
        u[c] = fields[c].transpose(2, 1, 0)
    p = lambda a: a.ctypes.data_as(D)
    L.step_host(w.words, w.n_r, w.n_theta, w.angular_order, p(ch), p(cf), p(wt), p(scal), p(u), nsteps)
    return [u[c].transpose(2, 1, 0) for c in range(4)]


@pytest.mark.parametrize("words,m,a,order", [(1, 2, 0.5, 10), (2, 2, 0.5, 10), (4, 2, 0.99, 10), (2, 1, 0.9, 10),
                                              (4, 0, 0.3, 2)])
def test_host_step_matches_oracle(words, m, a, order):
    w = inputs.C1.with_(n_r=33, n_theta=10, rstar_min=70.0, rstar_max=140.0, words=words, m=m, a_over_M=a,
                        angular_order=order)
    f = inputs.initial_fields(w)
    got = host_steps(w, f, 8)
    ref = oracle_run(w, f, 8)
    assert rel_linf(got, ref) <= TOL[words]
