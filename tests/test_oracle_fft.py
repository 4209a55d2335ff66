"""Pin P1: the oracle's radix-2 FFT equals the direct DFT (the definition),
and both agree with numpy.fft as an independent implementation."""
import numpy as np
import pytest

from oracle import fft


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128])
def test_radix2_equals_direct_dft(n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=(4, n)) + 1j * rng.normal(size=(4, n))
    a = fft.fft_radix2(x)
    b = fft.dft_direct(x)
    assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))
    ai = fft.fft_radix2(x, inverse=True)
    bi = fft.dft_direct(x, inverse=True)
    assert np.max(np.abs(ai - bi)) <= 1e-13 * max(1.0, np.max(np.abs(bi)))


def test_matches_numpy_fft_and_roundtrip():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(2, 8, 16, 32)) + 1j * rng.normal(size=(2, 8, 16, 32))
    X = fft.fft3(x)
    ref = np.fft.fftn(x, axes=(-3, -2, -1))
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref))
    back = fft.ifft3(X)
    assert np.max(np.abs(back - x)) <= 1e-13 * np.max(np.abs(x))


def test_direct_dft_non_power_of_two():
    rng = np.random.default_rng(3)
    for n in (3, 6, 12, 24, 48):
        x = rng.normal(size=n) + 1j * rng.normal(size=n)
        assert np.allclose(fft.dft_direct(x), np.fft.fft(x), rtol=0, atol=1e-12 * n)
        y = fft.transform_axis(x[None], -1)
        assert np.allclose(y[0], np.fft.fft(x), rtol=0, atol=1e-12 * n)


def test_single_tone_and_sign_convention():
    # forward transform uses exp(-i k r): x[n] = exp(+2 pi i 3 n / 16) -> X[3] = 16
    n = 16
    x = np.exp(2j * np.pi * 3 * np.arange(n) / n)
    X = fft.fft_radix2(x)
    expect = np.zeros(n, complex)
    expect[3] = n
    assert np.max(np.abs(X - expect)) < 1e-13


def test_parseval():
    rng = np.random.default_rng(11)
    x = rng.normal(size=64) + 1j * rng.normal(size=64)
    X = fft.fft_radix2(x)
    assert abs(np.sum(np.abs(X) ** 2) / 64 - np.sum(np.abs(x) ** 2)) < 1e-11
