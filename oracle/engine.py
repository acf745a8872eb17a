"""ctypes driver of the fixed-point C engine (test infrastructure).

``build()`` compiles fxp_engine.c with gcc (-O2, OpenMP) into
oracle/liboracle_fxp.so.  ``run()`` converts the >= 400-bit tables of
``oracle.problem.build_tables`` and the initial fields (float64 word
arrays: the exact sum of the words is the value) to 384-bit fixed point,
steps, and returns the fields as Python integers scaled by 2^-384.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fxp_engine.c")
LIB = os.path.join(HERE, "liboracle_fxp.so")
FRAC = 384
NL = 7
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-Werror", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        lib = ctypes.CDLL(LIB)
        p = ctypes.c_void_p
        lib.oracle_lw_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_int,
                                      ctypes.c_int, p, p, p, p, p, p, p, p]
        lib.oracle_lw_run.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        assert lib.oracle_fx_limbs() == NL and lib.oracle_fx_frac_bits() == FRAC
        _lib = lib
    return _lib


# ---------------------------------------------------------------- conversions
def round_scaled(x, bits: int) -> int:
    """Nearest integer to x * 2^bits, ties away from zero, computed exactly from
    the number's integer mantissa and exponent (x an mpf, Fraction, int or float).
    (mpmath's own routines would work at the context precision, 53 bits by
    default, and silently drop the low bits.)"""
    if isinstance(x, int):
        return x << bits
    if isinstance(x, float):
        x = Fraction(x)
    if isinstance(x, Fraction):
        n = abs(x.numerator) << bits
        q, r = divmod(n, x.denominator)
        q += 1 if 2 * r >= x.denominator else 0
        return -q if x.numerator < 0 else q
    # read the stored (sign, mantissa, exponent) directly: constructing or
    # scaling an mpf would round it to the ambient context precision
    sign, man, exp, bc = (x if isinstance(x, mp.mpf) else mp.mpf(x))._mpf_
    if man == 0 and (exp != 0 or bc != 0):
        raise ValueError("non-finite value")
    shift = exp + bits
    if shift >= 0:
        q = man << shift
    else:
        q, r = divmod(man, 1 << -shift)
        q += 1 if 2 * r >= (1 << -shift) else 0
    return -q if sign else q


def mp_to_fixed(x) -> int:
    """Nearest integer to x * 2^FRAC (x an mp number, Fraction or int)."""
    return round_scaled(x, FRAC)


def words_to_fixed(words) -> int:
    """Exact value of a sequence of float64 words (their sum), rounded to 2^-FRAC."""
    total = Fraction(0)
    for w in words:
        total += Fraction(float(w))
    return mp_to_fixed(total)


def ints_to_limbs(vals) -> np.ndarray:
    buf = b"".join(int(v).to_bytes(8 * NL, "little", signed=True) for v in vals)
    return np.frombuffer(buf, dtype="<u8").copy()


def limbs_to_ints(arr: np.ndarray) -> list:
    b = arr.astype("<u8").tobytes()
    s = 8 * NL
    return [int.from_bytes(b[k:k + s], "little", signed=True) for k in range(0, len(b), s)]


def tables_to_fixed(T, processes: int = 1):
    """Limb arrays for the engine from oracle.problem tables (mp numbers or Fractions)."""
    def flat_coef(grid):
        vals = []
        for row in grid:
            for pt in row:
                b, W, K, Ct, C0 = pt
                for z in (b, W):
                    vals.append(z)
                for z in (K, Ct, C0):
                    if isinstance(z, tuple):
                        vals.extend(z)
                    else:
                        vals.extend((z.real, z.imag))
        return vals

    def conv(vals):
        if processes > 1 and len(vals) > 20000:
            import multiprocessing as mproc
            with mproc.get_context("fork").Pool(processes) as pool:
                ints = pool.map(mp_to_fixed, vals, chunksize=2048)
        else:
            ints = [mp_to_fixed(v) for v in vals]
        return ints_to_limbs(ints)

    return {
        "half": conv(flat_coef(T["half"])),
        "full": conv(flat_coef(T["full"])),
        "cot": conv(T["cot"]), "V": conv(T["V"]),
        "d1": conv(T["d1"]), "d2": conv(T["d2"]),
        "scal": conv([T["inv_h"], T["dt"]]),
        "reach": T["reach"], "parity": T["parity"],
    }


def fields_to_fixed(fields) -> list:
    """fields: sequence of 4 arrays [nth][nr][p] (float64 words) -> flat list of ints [4][nth][nr]."""
    out = []
    for f in fields:
        a = np.asarray(f, dtype=np.float64)
        if a.ndim == 2:
            a = a[..., None]
        for w in a.reshape(-1, a.shape[-1]):
            out.append(words_to_fixed(w))
    return out


# ---------------------------------------------------------------- stepping
def run_fixed(FT, nr: int, nth: int, u_ints: list, nsteps: int, threads: int = 0) -> list:
    """Advance fixed-point state (flat ints [4][nth][nr]) by nsteps; returns ints."""
    lib = _load()
    if threads:
        lib.oracle_set_threads(int(threads))
    u = ints_to_limbs(u_ints)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.oracle_lw_run(nr, nth, nsteps, FT["reach"], FT["parity"], ptr(FT["half"]),
                           ptr(FT["full"]), ptr(FT["cot"]), ptr(FT["V"]), ptr(FT["d1"]),
                           ptr(FT["d2"]), ptr(FT["scal"]), ptr(u))
    if rc != 0:
        raise ArithmeticError("oracle engine failed with code %d" % rc)
    return limbs_to_ints(u)


def threads_in_use() -> int:
    """Threads the engine's parallel loops run on now."""
    return _load().oracle_set_threads(0)


def fixed_to_float(vals) -> np.ndarray:
    return np.array([v / (1 << FRAC) for v in vals], dtype=np.float64)


def run_problem(problem, fields, nsteps: int, processes: int = 1, tables=None):
    """Oracle evolution of ``fields`` (4 float64 word arrays [nth][nr][p]) for a
    ``oracle.problem.Problem``; returns flat ints [4][nth][nr] scaled 2^-FRAC."""
    from . import problem as _pb
    if tables is None:
        tables = _pb.build_tables(problem, processes=processes)
    FT = tables_to_fixed(tables, processes=processes)
    u = fields_to_fixed(fields)
    return run_fixed(FT, problem.n_r, problem.n_theta, u, nsteps, threads=processes)
