"""Python binding of libteuk (include/teuk.h): argument marshalling only.

Every entry point of the C ABI is available under its C name through
``lib()``; the ``Teuk`` and ``TeukBatch`` classes wrap a handle and raise
``TeukError`` on a negative return code.  Field arrays are numpy float64 in
the interchange layout [n_theta][n_r][words].  All stepping runs in the
library's gfx950 kernels; there is no Python or CPU fallback: if libteuk.so
has not been built this module raises on first use.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libteuk.so")

TEUK_OK, TEUK_EINVAL, TEUK_ENOMEM, TEUK_EDEVICE, TEUK_ENOTSUP, TEUK_ENONFINITE = 0, -1, -2, -3, -4, -5
FP64, DD, QD = 1, 2, 4
SWEEP_SEGMENT, SWEEP_WIDE, SWEEP_WIDE2, SWEEP_SLAB = 0, 1, 2, 3
PHI_RE, PHI_IM, PI_RE, PI_IM = 0, 1, 2, 3


class TeukError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libteuk error %d: %s" % (code, msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int), ("n_theta", ctypes.c_int), ("rstar_min", ctypes.c_double),
                ("rstar_max", ctypes.c_double), ("cfl", ctypes.c_double), ("mass", ctypes.c_double),
                ("angular_order", ctypes.c_int)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "teuk_abi_version": ([], ctypes.c_int),
    "teuk_build_info": ([], ctypes.c_char_p),
    "teuk_last_error": ([], ctypes.c_char_p),
    "teuk_validate": ([ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(Grid), ctypes.c_int], ctypes.c_int),
    "teuk_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(Grid), ctypes.c_int,
                     ctypes.POINTER(_P)], ctypes.c_int),
    "teuk_destroy": ([_P], ctypes.c_int),
    "teuk_set_initial": ([_P, _D, _D, _D, _D], ctypes.c_int),
    "teuk_step": ([_P, ctypes.c_long], ctypes.c_int),
    "teuk_read_field": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "teuk_dt": ([_P], ctypes.c_double),
    "teuk_steps_done": ([_P], ctypes.c_long),
    "teuk_words": ([_P], ctypes.c_int),
    "teuk_set_step_index": ([_P, ctypes.c_long], ctypes.c_int),
    "teuk_set_stream": ([_P, _P], ctypes.c_int),
    "teuk_check_finite": ([_P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "teuk_set_tile": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_set_launch": ([_P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "teuk_batch_set_launch": ([_P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "teuk_set_sweep": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_get_sweep": ([_P], ctypes.c_int),
    "teuk_batch_set_sweep": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_set_fuse": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_batch_set_fuse": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_get_coefficients": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "teuk_set_coefficients": ([_P, ctypes.c_int, _D], ctypes.c_int),
    "teuk_batch_create": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _D,
                           ctypes.POINTER(Grid), ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "teuk_batch_destroy": ([_P], ctypes.c_int),
    "teuk_batch_set_initial": ([_P, ctypes.c_int, _D, _D, _D, _D], ctypes.c_int),
    "teuk_batch_step": ([_P, ctypes.c_long], ctypes.c_int),
    "teuk_batch_read_field": ([_P, ctypes.c_int, ctypes.c_int, _D], ctypes.c_int),
    "teuk_batch_set_stream": ([_P, _P], ctypes.c_int),
    "teuk_batch_size": ([_P], ctypes.c_int),
    "teuk_batch_dt": ([_P, ctypes.c_int], ctypes.c_double),
    "teuk_batch_set_tile": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_batch_use_graph": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_use_graph": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_prepare_graph": ([_P], ctypes.c_int),
    "teuk_batch_prepare_graph": ([_P], ctypes.c_int),
    "teuk_graph_replays": ([_P], ctypes.c_long),
    "teuk_batch_graph_replays": ([_P], ctypes.c_long),
    "teuk_set_host_round_trip": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_batch_set_host_round_trip": ([_P, ctypes.c_int], ctypes.c_int),
    "teuk_set_observer": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                           ctypes.c_int, ctypes.c_long], ctypes.c_int),
    "teuk_read_observer": ([_P, ctypes.c_long, _D, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)],
                           ctypes.c_int),
    "teuk_coefficients_noalloc": ([ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(Grid), ctypes.c_int,
                                   _P, _P, _P, _P], ctypes.c_int),
    "teuk_fp64_fma_probe": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _D, _D], ctypes.c_int),
    "teuk_arith_host": ([ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_int], ctypes.c_int),
    "teuk_arith_device": ([ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_int], ctypes.c_int),
}
_lib = None


def lib():
    """The loaded libteuk.so with every C entry point typed; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libteuk.so is not built (python -m paper_1006_0663_amd.build); "
                               "there is no fallback implementation")
        # PyTorch ships its own HIP runtime under a different file name; loaded
        # first, it also serves this library (same soname), so the process holds
        # one runtime and torch's streams and device pointers are valid here.
        # Loaded after this library, torch would start a second runtime that
        # finds no GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != TEUK_OK:
        raise TeukError(rc, lib().teuk_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_D)


def make_grid(n_r, n_theta, rstar_min, rstar_max, cfl=0.5, mass=1.0, angular_order=10):
    return Grid(n_r, n_theta, rstar_min, rstar_max, cfl, mass, angular_order)


def _field_array(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        a = a.reshape(shape)
    return a


class Teuk:
    """One Teukolsky instance on the current GPU (wraps a teuk_t handle)."""

    def __init__(self, s, m, a_over_M, grid: Grid, words: int):
        self.grid, self.words = grid, words
        h = _P()
        _check(lib().teuk_create(s, m, a_over_M, ctypes.byref(grid), words, ctypes.byref(h)))
        self.h = h
        self.shape = (grid.n_theta, grid.n_r, words)

    def close(self):
        if getattr(self, "h", None):
            lib().teuk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_initial(self, phi_re, phi_im, pi_re, pi_im):
        arrs = [_field_array(x, self.shape) for x in (phi_re, phi_im, pi_re, pi_im)]
        _check(lib().teuk_set_initial(self.h, *[_dptr(x) for x in arrs]))

    def step(self, n):
        _check(lib().teuk_step(self.h, int(n)))

    def read_field(self, f):
        out = np.empty(self.shape)
        _check(lib().teuk_read_field(self.h, f, _dptr(out)))
        return out

    def fields(self):
        return tuple(self.read_field(f) for f in range(4))

    def _handle(self):
        if not getattr(self, "h", None):
            raise TeukError(TEUK_EINVAL, "handle is closed")
        return self.h

    @property
    def dt(self):
        return lib().teuk_dt(self._handle())

    @property
    def steps_done(self):
        return lib().teuk_steps_done(self._handle())

    def set_step_index(self, n):
        _check(lib().teuk_set_step_index(self.h, int(n)))

    def set_stream(self, stream_ptr):
        _check(lib().teuk_set_stream(self.h, _P(stream_ptr or 0)))

    def set_tile(self, segcols):
        _check(lib().teuk_set_tile(self.h, int(segcols)))

    def set_launch(self, segcols, block=0):
        _check(lib().teuk_set_launch(self.h, int(segcols), int(block)))

    def use_graph(self, k):
        _check(lib().teuk_use_graph(self.h, int(k)))

    def set_sweep(self, sweep):
        _check(lib().teuk_set_sweep(self.h, int(sweep)))

    def prepare_graph(self):
        _check(lib().teuk_prepare_graph(self.h))

    @property
    def graph_replays(self):
        return lib().teuk_graph_replays(self.h)

    def set_host_round_trip(self, on):
        _check(lib().teuk_set_host_round_trip(self.h, int(bool(on))))

    def set_observer(self, points, every=1, capacity=1 << 16):
        """points: sequence of (i, j) grid indices (r* node, theta row); [] removes the observer."""
        n = len(points)
        ii = (ctypes.c_int * max(n, 1))(*[int(p[0]) for p in points])
        jj = (ctypes.c_int * max(n, 1))(*[int(p[1]) for p in points])
        _check(lib().teuk_set_observer(self.h, n, ii, jj, int(every), int(capacity)))
        self._obs = (n, int(capacity))

    def read_observer(self, max_records=None):
        """(steps [n], phi [n][points][2][words], records written since set_initial)."""
        npts, cap = self._obs
        k = cap if max_records is None else int(max_records)
        rec = 1 + 2 * self.words * npts
        out = np.empty((max(k, 1), rec))
        n_out, n_tot = ctypes.c_long(0), ctypes.c_long(0)
        _check(lib().teuk_read_observer(self.h, k, _dptr(out), ctypes.byref(n_out), ctypes.byref(n_tot)))
        out = out[:n_out.value]
        return out[:, 0].astype(np.int64), out[:, 1:].reshape(-1, npts, 2, self.words), n_tot.value

    @property
    def sweep(self):
        return lib().teuk_get_sweep(self.h)

    def set_fuse(self, steps_per_launch):
        _check(lib().teuk_set_fuse(self.h, int(steps_per_launch)))

    def check_finite(self):
        ok = ctypes.c_int(0)
        rc = lib().teuk_check_finite(self.h, ctypes.byref(ok))
        if rc not in (TEUK_OK, TEUK_ENONFINITE):
            _check(rc)
        return bool(ok.value)

    def coefficients(self, which):
        nth, nr, W = self.grid.n_theta, self.grid.n_r, self.words
        if which == 2:
            R = self.grid.angular_order // 2
            out = np.empty((2 * R + 1, nth, W))
        else:
            out = np.empty((8, nth, nr - 1 if which == 0 else nr, W))
        _check(lib().teuk_get_coefficients(self.h, which, _dptr(out)))
        return out

    def set_coefficients(self, which, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        _check(lib().teuk_set_coefficients(self.h, which, _dptr(arr)))


class TeukBatch:
    """Many independent instances advanced together (wraps a teuk_batch_t handle)."""

    def __init__(self, specs, words):
        """specs: sequence of (s, m, a_over_M, Grid)."""
        n = len(specs)
        s = (ctypes.c_int * n)(*[x[0] for x in specs])
        m = (ctypes.c_int * n)(*[x[1] for x in specs])
        a = (ctypes.c_double * n)(*[x[2] for x in specs])
        g = (Grid * n)(*[x[3] for x in specs])
        h = _P()
        _check(lib().teuk_batch_create(n, s, m, a, g, words, ctypes.byref(h)))
        self.h, self.words = h, words
        self.grids = [x[3] for x in specs]

    def close(self):
        if getattr(self, "h", None):
            lib().teuk_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, k):
        g = self.grids[k]
        return (g.n_theta, g.n_r, self.words)

    def set_initial(self, k, phi_re, phi_im, pi_re, pi_im):
        arrs = [_field_array(x, self.shape(k)) for x in (phi_re, phi_im, pi_re, pi_im)]
        _check(lib().teuk_batch_set_initial(self.h, k, *[_dptr(x) for x in arrs]))

    def step(self, n):
        _check(lib().teuk_batch_step(self.h, int(n)))

    def read_field(self, k, f):
        out = np.empty(self.shape(k))
        _check(lib().teuk_batch_read_field(self.h, k, f, _dptr(out)))
        return out

    def dt(self, k):
        return lib().teuk_batch_dt(self.h, k)

    def set_stream(self, stream_ptr):
        _check(lib().teuk_batch_set_stream(self.h, _P(stream_ptr or 0)))

    def set_tile(self, segcols):
        _check(lib().teuk_batch_set_tile(self.h, int(segcols)))

    def set_launch(self, segcols, block=0):
        _check(lib().teuk_batch_set_launch(self.h, int(segcols), int(block)))

    def set_sweep(self, sweep):
        _check(lib().teuk_batch_set_sweep(self.h, int(sweep)))

    def set_fuse(self, steps_per_launch):
        _check(lib().teuk_batch_set_fuse(self.h, int(steps_per_launch)))

    def use_graph(self, k):
        _check(lib().teuk_batch_use_graph(self.h, int(k)))

    def prepare_graph(self):
        _check(lib().teuk_batch_prepare_graph(self.h))

    @property
    def graph_replays(self):
        return lib().teuk_batch_graph_replays(self.h)

    def set_host_round_trip(self, on):
        _check(lib().teuk_batch_set_host_round_trip(self.h, int(bool(on))))


def arith(words, op, a, b, device=False):
    """Apply one multiword operation to arrays a, b of shape [n][words]."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, words)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1, words)
    out = np.empty_like(a)
    f = lib().teuk_arith_device if device else lib().teuk_arith_host
    _check(f(words, op, _dptr(a), _dptr(b), _dptr(out), a.shape[0]))
    return out


def fp64_fma_probe(chains, blocks, threads, iters):
    """(TFLOP/s, ms) of the FP64 FMA probe kernel (see teuk_fp64_fma_probe)."""
    tf, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().teuk_fp64_fma_probe(int(chains), int(blocks), int(threads), int(iters), ctypes.byref(tf),
                                   ctypes.byref(ms))
    if rc != TEUK_OK:
        raise TeukError(rc, "fp64 FMA probe failed")
    return tf.value, ms.value


def coefficients_noalloc(s, m, a_over_M, grid: Grid, words, d_ch, d_cf, d_wt, stream=0):
    """Coefficient pass into caller-owned device buffers (addresses as ints)
    on `stream` (a hipStream_t as int); see teuk_coefficients_noalloc."""
    _check(lib().teuk_coefficients_noalloc(s, m, a_over_M, ctypes.byref(grid), words, _P(d_ch), _P(d_cf),
                                           _P(d_wt), _P(stream or 0)))
