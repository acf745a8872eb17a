"""Pins of oracle.stencils: published tables, textbook stencils, convergence order."""
from fractions import Fraction as F
import math

import mpmath as mp

from oracle.stencils import central_weights


def test_second_order_textbook():
    assert central_weights(1, 1) == [F(-1, 2), F(0), F(1, 2)]
    assert central_weights(2, 1) == [F(1), F(-2), F(1)]


def test_tenth_order_published_table():
    # Fornberg (1988), Table 1: centred weights, accuracy order 10
    d1 = [F(5, 6), F(-5, 21), F(5, 84), F(-5, 504), F(1, 1260)]
    d2 = [F(5, 3), F(-5, 21), F(5, 126), F(-5, 1008), F(1, 3150)]
    c1, c2 = central_weights(1, 5), central_weights(2, 5)
    assert c1[5] == 0 and c1[6:] == d1 and c1[:5] == [-x for x in reversed(d1)]
    assert c2[5] == F(-5269, 1800) and c2[6:] == d2 and c2[:5] == list(reversed(d2))


def test_tenth_order_convergence_on_sin():
    with mp.workprec(300):
        c1, c2 = central_weights(1, 5), central_weights(2, 5)
        x0 = mp.mpf("0.7")
        errs = []
        for h in (mp.mpf(1) / 8, mp.mpf(1) / 16):
            v1 = sum(mp.mpf(c.numerator) / c.denominator * mp.sin(x0 + k * h) for k, c in zip(range(-5, 6), c1)) / h
            v2 = sum(mp.mpf(c.numerator) / c.denominator * mp.sin(x0 + k * h) for k, c in zip(range(-5, 6), c2)) / h ** 2
            errs.append((abs(v1 - mp.cos(x0)), abs(v2 + mp.sin(x0))))
        for a, b in zip(errs[0], errs[1]):
            order = math.log2(float(a / b))
            assert 9.7 < order < 10.3, order
