"""Discrete Fourier transforms for the oracle (test infrastructure only).

The paper replaces the continuous Fourier transform on the box D by its
discrete counterpart on the uniform grid and evaluates it with the FFT
(Sec. 2, discretisation paragraph).  Sign convention of the forward
transform: exp(-i k.r), as in the paper's definition of F(G) (Sec. 2, text
before Eq. 7).  The inverse carries the 1/N factor.

Two independent implementations:
  dft_direct  the definition X[m] = sum_n x[n] exp(-2 pi i m n / N), O(N^2)
  fft_radix2  iterative radix-2 decimation-in-time Cooley-Tukey, N = 2^p
Test pin: fft_radix2 == dft_direct to round-off for N = 2..64 (tests).
"""
import numpy as np


def _twiddle(n_total, idx, sign):
    """exp(sign * 2 pi i * idx / n_total) with idx reduced mod n_total first,
    so that large products m*n keep full accuracy."""
    idx = np.mod(idx, n_total)
    return np.exp(sign * 2j * np.pi * idx / n_total)


def dft_direct(x, inverse=False):
    """Direct DFT along the last axis: the definition, O(N^2) per transform.

    forward: X[m] = sum_n x[n] exp(-2 pi i m n / N)
    inverse: x[n] = (1/N) sum_m X[m] exp(+2 pi i m n / N)
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    sign = 1.0 if inverse else -1.0
    mn = np.outer(np.arange(n), np.arange(n))
    w = _twiddle(n, mn, sign)                     # w[m, k]
    y = x @ w.T                                   # y[..., m] = sum_k x[..., k] w[m, k]
    if inverse:
        y = y / n
    return y


def _bit_reverse(n):
    bits = n.bit_length() - 1
    rev = np.zeros(n, dtype=np.int64)
    for i in range(n):
        r, v = 0, i
        for _ in range(bits):
            r = (r << 1) | (v & 1)
            v >>= 1
        rev[i] = r
    return rev


def fft_radix2(x, inverse=False):
    """Iterative radix-2 DIT FFT along the last axis (length a power of two).

    Input is permuted to bit-reversed order; then for sub-transform sizes
    2, 4, ..., N each pair (even half E, odd half O) of length size/2 is
    combined as  E + w^k O,  E - w^k O  with w = exp(-+ 2 pi i / size).
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    if n < 1 or (n & (n - 1)) != 0:
        raise ValueError("fft_radix2 needs a power-of-two length, got %d" % n)
    sign = 1.0 if inverse else -1.0
    lead = x.shape[:-1]
    a = x[..., _bit_reverse(n)]
    size = 2
    while size <= n:
        half = size // 2
        w = _twiddle(size, np.arange(half), sign)
        a = a.reshape(lead + (n // size, size))
        even = a[..., :half]
        odd = a[..., half:] * w
        a = np.concatenate([even + odd, even - odd], axis=-1)
        size *= 2
    a = a.reshape(lead + (n,))
    if inverse:
        a = a / n
    return a


def transform_axis(x, axis, inverse=False):
    """1D transform along one axis: radix-2 for powers of two, else direct."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    if n & (n - 1) == 0:
        y = fft_radix2(x, inverse)
    else:
        y = dft_direct(x, inverse)
    return np.moveaxis(y, -1, axis)


def fft3(v):
    """Forward 3D DFT over the last three axes (z, y, x)."""
    y = np.asarray(v, dtype=np.complex128)
    for ax in (-1, -2, -3):
        y = transform_axis(y, ax, inverse=False)
    return y


def ifft3(v):
    """Inverse 3D DFT over the last three axes, with the 1/(Nx Ny Nz) factor."""
    y = np.asarray(v, dtype=np.complex128)
    for ax in (-1, -2, -3):
        y = transform_axis(y, ax, inverse=True)
    return y


def dft3_direct(v, inverse=False):
    """3D DFT by the direct definition applied along each axis (no FFT)."""
    y = np.asarray(v, dtype=np.complex128)
    for ax in (-1, -2, -3):
        y = np.moveaxis(dft_direct(np.moveaxis(y, ax, -1), inverse), -1, ax)
    return y
