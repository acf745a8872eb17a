"""Centred finite-difference weights, exact rationals (test infrastructure).

The paper evaluates angular derivatives with centred differences: second
order in the base scheme (Sec. "Teukolsky Code") and tenth order in the
production runs (Sec. "High-Order and High-Precision").  A centred stencil of
reach R (2R+1 points) of maximal order for the d-th derivative is *defined*
by requiring it to be exact on every polynomial of degree <= 2R:

    sum_{k=-R..R} c_k k^p = d! * [p == d],   p = 0..2R.

This module solves that Vandermonde system exactly over the rationals.
Pins: the published 10th-order table values and the textbook 2nd-order
stencils (tests/test_oracle_stencils.py), plus the observed convergence
order on sin(x).
"""
from fractions import Fraction
from math import factorial


def central_weights(deriv: int, reach: int) -> list:
    """Weights c_{-R..R} (list of Fraction, index k+R) for d^deriv/dx^deriv.

    The derivative at x_j on a unit-spaced grid is sum_k c_k f(x_{j+k});
    for spacing h divide by h**deriv.
    """
    if reach < 1 or deriv < 0 or deriv > 2 * reach:
        raise ValueError("need reach >= 1 and 0 <= deriv <= 2*reach")
    n = 2 * reach + 1
    offsets = list(range(-reach, reach + 1))
    # augmented matrix rows: p-th moment condition
    a = [[Fraction(k) ** p for k in offsets] + [Fraction(factorial(deriv)) if p == deriv else Fraction(0)]
         for p in range(n)]
    # Gauss-Jordan elimination, exact
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        inv = 1 / a[col][col]
        a[col] = [v * inv for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [vr - f * vc for vr, vc in zip(a[r], a[col])]
    return [a[r][n] for r in range(n)]


def angular_reach(order: int) -> int:
    """Stencil reach for an even order of accuracy (2 -> 1, 10 -> 5)."""
    if order < 2 or order % 2:
        raise ValueError("angular order must be even and >= 2")
    return order // 2
