"""The library FFT used by the oracle against the brute-force DFT definition."""
import numpy as np
import pytest

from oracle import dft_direct


@pytest.mark.parametrize("shape", [(8, 9, 10), (5, 6, 4), (9, 9, 9), (3, 12, 5), (20, 4, 2)])
def test_fftn_vs_direct(shape):
    rng = np.random.default_rng(sum(shape))
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np.testing.assert_allclose(np.fft.fftn(f), dft_direct.dft3(f, -1), rtol=0, atol=1e-10 * np.abs(f).sum())
    np.testing.assert_allclose(np.fft.ifftn(f) * f.size, dft_direct.dft3(f, +1), rtol=0,
                               atol=1e-10 * np.abs(f).sum())


def test_single_mode_is_plane_wave():
    shape = (6, 5, 4)
    c = np.zeros(shape, complex)
    m = (2, 4, 1)
    c[m] = 1.0
    r = dft_direct.dft3(c, +1)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1)
    expect = np.exp(2j * np.pi * (j[..., 0] * m[0] / 6 + j[..., 1] * m[1] / 5 + j[..., 2] * m[2] / 4))
    np.testing.assert_allclose(r, expect, atol=1e-13)


def test_parseval():
    rng = np.random.default_rng(7)
    f = rng.standard_normal((10, 6, 9)) + 1j * rng.standard_normal((10, 6, 9))
    F = dft_direct.dft3(f)
    assert abs((np.abs(f) ** 2).sum() - (np.abs(F) ** 2).sum() / f.size) < 1e-10 * (np.abs(f) ** 2).sum()
