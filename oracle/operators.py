"""Spectral operators on a periodic grid (test infrastructure only).

C_s, the smoothed spectral curl (Sec. 2: derivatives in Eqs. 3 and 4 are taken
in Fourier space with Gaussian smoothing):
    C_s v = Re F^-1 { S(k) * i k_odd x F(v) }
Phi, the Biot-Savart operator (Eq. 7, with the rule of the k = 0 paragraph
after it: 1/|k|^2 is replaced by 0 at k = 0):
    Phi[j] = Re F^-1 { i k_odd x F(j) / |k|^2 },   0 at k = 0
By default Phi is not smoothed (the paper smooths only the derivatives in
Eqs. 3 and 4); smooth_phi=True multiplies its symbol by S(k) as well.
Also: div_s (smoothed spectral divergence, used by tests for div j = 0) and
the Leray projector (used by tests: curl Phi[j] = S P j).
F is this package's own FFT (oracle.fft).
"""
import numpy as np

from . import fft as _fft


def _cross(ax, ay, az, bx, by, bz):
    """Componentwise a x b."""
    return (ay * bz - az * by, az * bx - ax * bz, ax * by - ay * bx)


def spectrum(v):
    """F of a vector field [3, z, y, x] (complex128)."""
    return _fft.fft3(v)


def real_field(V):
    """Re F^-1 of a vector spectrum."""
    return np.real(_fft.ifft3(V))


def curl_s(v, grid, sign=1.0):
    """sign * C_s v for a real vector field v of shape (3, Nz, Ny, Nx)."""
    V = spectrum(v)
    kx, ky, kz = grid.mesh_k(odd=True)
    s = grid.smoothing()
    cx, cy, cz = _cross(kx, ky, kz, V[0], V[1], V[2])
    out = np.stack([1j * cx, 1j * cy, 1j * cz]) * (sign * s)
    return real_field(out)


def phi(j, grid, smooth=False):
    """Phi[j]: the discrete Biot-Savart operator of Eq. 7 on the periodic box."""
    J = spectrum(j)
    kx, ky, kz = grid.mesh_k(odd=True)
    k2 = grid.k2()
    inv = np.zeros_like(k2)
    nz = k2 != 0.0
    inv[nz] = 1.0 / k2[nz]                         # k = 0 rule: 1/|k|^2 -> 0
    if smooth:
        inv = inv * grid.smoothing()
    cx, cy, cz = _cross(kx, ky, kz, J[0], J[1], J[2])
    out = np.stack([1j * cx, 1j * cy, 1j * cz]) * inv
    return real_field(out)


def div_s(v, grid):
    """Smoothed spectral divergence Re F^-1 { S i k_odd . F(v) }."""
    V = spectrum(v)
    kx, ky, kz = grid.mesh_k(odd=True)
    s = grid.smoothing()
    d = 1j * (kx * V[0] + ky * V[1] + kz * V[2]) * s
    return np.real(_fft.ifft3(d))


def leray(v, grid):
    """Divergence-free projection P v = v - k (k . v)/|k|^2 using k_odd in the
    projection and true |k_odd|^2 in the denominator (0 where k_odd = 0)."""
    V = spectrum(v)
    kx, ky, kz = grid.mesh_k(odd=True)
    k2o = kx * kx + ky * ky + kz * kz
    inv = np.zeros_like(k2o)
    nz = k2o != 0.0
    inv[nz] = 1.0 / k2o[nz]
    kv = (kx * V[0] + ky * V[1] + kz * V[2]) * inv
    out = np.stack([V[0] - kx * kv, V[1] - ky * kv, V[2] - kz * kv])
    return real_field(out)
