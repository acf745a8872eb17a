"""The seeded input generator (shared by the oracle and the library runs):
the l-projected compactly supported profile against closed forms."""
import mpmath as mp
import numpy as np
import pytest

from paper_1006_0663_amd import inputs


@pytest.mark.parametrize("ell,m", [(0, 0), (1, 0), (2, 1), (3, 2)])
def test_bump_legendre_profile(ell, m):
    """Phi(0) = (1 - x^2)^8 P_l^|m|(cos theta), x = (r* - r0)/(4 sigma): zero
    outside |x| < 1 and at the radial boundary nodes, Pi = 0, and the angular
    factor equal to the closed-form P_l^m (Condon-Shortley phase)."""
    closed = {(0, 0): lambda c, s: 1, (1, 0): lambda c, s: c,
              (2, 1): lambda c, s: -3 * c * s, (3, 2): lambda c, s: 15 * c * s * s}
    w = inputs.S0_KERR.with_(n_r=81, n_theta=12, rstar_min=30.0, rstar_max=110.0, m=m, ell=ell, words=2)
    pulse = inputs.Pulse(70.0, 5.0, 1.0, 0.0)
    f = inputs.initial_fields(w, pulse)
    assert np.all(f[2] == 0) and np.all(f[3] == 0) and np.all(f[1] == 0)
    rs = np.linspace(30.0, 110.0, 81)
    x = (rs - 70.0) / 20.0
    outside = np.abs(x) >= 1
    assert np.all(f[0][:, outside, :] == 0)
    assert np.all(f[0][:, [0, -1], :] == 0)
    i = 40                                    # r* = 70: bump = 1
    with mp.workprec(200):
        for j in range(w.n_theta):
            th = (j + mp.mpf(1) / 2) * mp.pi / w.n_theta
            want = closed[(ell, m)](mp.cos(th), mp.sin(th))
            got = mp.mpf(float(f[0][j, i, 0])) + mp.mpf(float(f[0][j, i, 1]))
            assert abs(got - want) <= mp.mpf(2) ** -100 * max(1, abs(want)), (j, got, want)
    k = 45                                    # r* = 75: (1 - 1/16)^8
    assert abs(f[0][0, k, 0] / f[0][0, i, 0] - (1 - 1 / 16) ** 8) < 1e-14


def test_l_projection_needs_spin_weight_zero():
    with pytest.raises(ValueError):
        inputs.initial_fields(inputs.S0_KERR.with_(s=-2, n_r=20, n_theta=8))
    with pytest.raises(ValueError):
        inputs.initial_fields(inputs.S0_KERR.with_(ell=0, m=1, n_r=20, n_theta=8))
