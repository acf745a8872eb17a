"""FP64 operations per grid-point update of the step kernel, counted from its
code (an FMA counts 2, every add/sub/mul 1; exact power-of-two scalings
count 1 per word).  Used to express throughput as a fraction of the FP64
vector peak.

Per update: two angular stencils (2 components x 11 products + result each)
and two stages; a stage forms 5 complex neighbour sums/differences (Phi, Pi
averages and differences, and the average of the two stencil values) with 6
real halvings, then four fused dot products: the two Phi outputs take 1 value
+ 2 products, the two Pi outputs 1 value + 8 products.  The FP64 kernel also
rebuilds its 8 coefficients at 2 locations per update (32 operations each).
"""

# cost of one fused-dot operation, by words per real
PROD = {1: 2, 2: 15, 4: 122}        # acc += a*b
VALUE = {1: 1, 2: 8, 4: 40}         # acc += v
RESULT = {1: 0, 2: 6, 4: 55}        # final normalisation
ADD_FAST = {1: 1, 2: 11, 4: 106}    # neighbour sum / difference
HALVE = {1: 1, 2: 2, 4: 4}
COEF_PER_POINT_FP64 = 32


def flops_per_update(words: int, taps: int = 11, onfly_fp64: bool = True) -> int:
    stencil = 2 * (taps * PROD[words] + RESULT[words])
    stage = (10 * ADD_FAST[words] + 6 * HALVE[words]
             + 2 * (VALUE[words] + 2 * PROD[words] + RESULT[words])
             + 2 * (VALUE[words] + 8 * PROD[words] + RESULT[words]))
    total = 2 * stencil + 2 * stage
    if words == 1 and onfly_fp64:
        total += 2 * COEF_PER_POINT_FP64
    return total


def bytes_per_update(words: int, onfly_fp64: bool = True) -> int:
    """Algorithmic HBM bytes per update: state read + state write, plus the
    16 stored coefficients unless the FP64 kernel rebuilds them per point."""
    coef = 0 if (words == 1 and onfly_fp64) else 16
    return (4 + 4 + coef) * 8 * words
