"""Pins of the oracle's Fourier transforms (pin T1).

The radix-2 FFT (and the mixed-radix transform used for lengths such as the
N = 180 * 2^k of Example 1) is checked against the O(N^2) DFT written out, against
numpy's FFT (an independent library routine), and against identities of the
DFT (inverse, Parseval, a single mode maps to a delta).  The sign convention
is the one of the paper's Fourier transform (Eqn. FT): exp(-i x.xi) forward.
"""
import numpy as np
import pytest

from tests.util import rel


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64])
def test_radix2_matches_naive_dft(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, +1):
        assert rel(orc.fft1d(x, sign), orc.dft1d_naive(x, sign)) < 1e-13


@pytest.mark.parametrize("n", [2, 64, 1024])
def test_radix2_matches_numpy(orc, n):
    rng = np.random.default_rng(n + 1)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert rel(orc.fft1d(x, -1), np.fft.fft(x)) < 1e-13
    assert rel(orc.fft1d(x, +1), np.fft.ifft(x) * n) < 1e-13


def test_single_mode_is_delta(orc):
    n, k = 32, 5
    j = np.arange(n)
    x = np.exp(2j * np.pi * k * j / n)        # exp(+i xi x) at xi = 2 pi k
    X = orc.fft1d(x, -1)
    e = np.zeros(n, complex)
    e[k] = n
    assert np.abs(X - e).max() < 1e-12


@pytest.mark.parametrize("shape", [(8, 16), (16, 16), (4, 8, 16)])
def test_nd_roundtrip_parseval_numpy(orc, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    X = orc.fftnd(x)
    assert rel(X, np.fft.fftn(x)) < 1e-13
    assert rel(orc.fftnd(X, inverse=True), x) < 1e-14
    assert abs(np.vdot(X, X).real / x.size - np.vdot(x, x).real) < 1e-12 * np.vdot(x, x).real


def test_nd_axis_order(orc):
    """A mode along the last axis must land on the last index (catches a transposed axis)."""
    n0, n1 = 8, 16
    i0, i1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    x = np.exp(2j * np.pi * (1 * i0 / n0 + 3 * i1 / n1))
    X = orc.fftnd(x)
    assert abs(X[1, 3] - n0 * n1) < 1e-10
    X[1, 3] = 0
    assert np.abs(X).max() < 1e-10


@pytest.mark.parametrize("n", [3, 6, 7, 12, 15, 30, 45, 60, 90, 180])
def test_mixed_radix_matches_naive_dft(orc, n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, +1):
        assert rel(orc.fft1d(x, sign), orc.dft1d_naive(x, sign)) < 1e-13


@pytest.mark.parametrize("n", [360, 2400])
def test_mixed_radix_matches_numpy(orc, n):
    rng = np.random.default_rng(n + 3)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert rel(orc.fft1d(x, -1), np.fft.fft(x)) < 1e-13
    assert rel(orc.fft1d(x, +1), np.fft.ifft(x) * n) < 1e-13


@pytest.mark.parametrize("shape", [(12, 30), (20, 18, 10)])
def test_mixed_radix_nd_matches_numpy(orc, shape):
    rng = np.random.default_rng(sum(shape) + 7)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    X = orc.fftnd(x)
    assert rel(X, np.fft.fftn(x)) < 1e-13
    assert rel(orc.fftnd(X, inverse=True), x) < 1e-14
