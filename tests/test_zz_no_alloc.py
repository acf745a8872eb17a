"""teuk_coefficients_noalloc: the coefficient pass into caller-owned device
buffers with the library's static scratch, against teuk_get_coefficients of
a handle created with the same arguments (same kernels: bitwise), on two
calls in a row per precision, the second on a smaller grid, and its size
limit."""
import numpy as np
import pytest

from paper_1006_0663_amd import teuk as T

pytestmark = pytest.mark.gpu


def _noalloc(torch, s, m, a, g, words, stream):
    nr, nth, R = g.n_r, g.n_theta, g.angular_order // 2
    ch = torch.full((8 * words * (nr - 1) * nth,), float("nan"), dtype=torch.float64, device="cuda")
    cf = torch.full((8 * words * nr * nth,), float("nan"), dtype=torch.float64, device="cuda")
    wt = torch.full(((2 * R + 1) * words * nth,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    T.coefficients_noalloc(s, m, a, g, words, ch.data_ptr(), cf.data_ptr(), wt.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    # device planar [c][w][i][j] -> interchange [c][j][i][w]
    half = ch.cpu().numpy().reshape(8, words, nr - 1, nth).transpose(0, 3, 2, 1)
    full = cf.cpu().numpy().reshape(8, words, nr, nth).transpose(0, 3, 2, 1)
    wts = wt.cpu().numpy().reshape(2 * R + 1, words, nth).transpose(0, 2, 1)
    return half, full, wts


def _handle(s, m, a, g, words):
    h = T.Teuk(s, m, a, g, words)
    out = (h.coefficients(0), h.coefficients(1), h.coefficients(2))
    h.close()
    return out


@pytest.mark.parametrize("words", [1, 2, 4])
def test_noalloc_coefficients_equal_the_handles(words):
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    cases = [(-2, 2, 0.9, T.make_grid(300, 64, -200.0, 800.0, 0.15)),
             (0, 1, 0.5, T.make_grid(37, 12, 20.0, 90.0, 0.3, angular_order=2))]   # second call: smaller grid
    for s, m, a, g in cases:
        print("noalloc coefficients words=%d s=%d m=%d a=%.2f %dx%d" % (words, s, m, a, g.n_r, g.n_theta),
              flush=True)
        got = _noalloc(torch, s, m, a, g, words, stream)
        ref = _handle(s, m, a, g, words)
        for k in range(3):
            assert got[k].shape == ref[k].shape, k
            assert np.array_equal(got[k], ref[k]), (words, k)


def test_noalloc_rejects_grids_beyond_its_scratch():
    import torch
    torch.cuda.set_device(0)
    L = T.lib()
    big = T.make_grid(40000, 256, -200.0, 800.0, 0.15)       # FP64 needs ~1.28e6 doubles of scratch
    p = T._P(1)                                              # never dereferenced: refused before any device work
    assert L.teuk_coefficients_noalloc(-2, 2, 0.5, big, 1, p, p, p, None) == T.TEUK_EINVAL
    assert "scratch" in L.teuk_last_error().decode()
    assert L.teuk_coefficients_noalloc(-2, 2, 0.5, big, 1, None, p, p, None) == T.TEUK_EINVAL
