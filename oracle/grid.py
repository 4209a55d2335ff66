"""Uniform node grid on the computational box and its wavenumbers.

Sec. 2 (discretisation paragraph): a uniform Nx x Ny x Nz grid is defined on
D = {|x| <= Lx, |y| <= Ly, |z| <= Lz}, the Fourier transform is replaced by
the DFT on that grid, derivatives are taken in Fourier space with Gaussian
smoothing whose parameter sigma is half of the grid-cell diagonal.

Readings where the paper is silent (each is listed in the design notes):
  * nodes are cell-centred: x_i = -L + (i + 1/2) * 2L/N, i = 0..N-1, so the
    DFT period is the box length 2L and k = pi * m / L for integer m;
  * m runs over 0..N/2-1, -N/2..-1 (the usual DFT order); for even N the
    Nyquist index m = -N/2 keeps its true k in |k|^2 and in the smoothing,
    but odd (first-derivative / cross-product) factors use k_odd, which is
    k with the Nyquist entry set to 0, so real fields stay real;
  * Gaussian smoothing multiplier S(k) = exp(-sigma^2 |k|^2 / 2) (sigma is
    the standard deviation of a unit-mass Gaussian kernel).
Arrays are laid out [z, y, x] with x fastest; vector fields are [3, z, y, x]
with components ordered (x, y, z).
"""
import numpy as np


class Grid:
    def __init__(self, n, half_width, sigma_scale=1.0):
        self.n = tuple(int(v) for v in n)             # (Nx, Ny, Nz)
        self.L = tuple(float(v) for v in half_width)  # (Lx, Ly, Lz), dimensionless
        for v in self.n:
            if v < 2 or v % 2:
                raise ValueError("grid counts must be even and >= 2")
        self.h = tuple(2.0 * L / N for L, N in zip(self.L, self.n))
        self.cell_volume = self.h[0] * self.h[1] * self.h[2]
        self.sigma = 0.5 * np.sqrt(self.h[0] ** 2 + self.h[1] ** 2 + self.h[2] ** 2) * sigma_scale

    @property
    def shape(self):
        """Scalar array shape (Nz, Ny, Nx)."""
        return (self.n[2], self.n[1], self.n[0])

    def axis_nodes(self, a):
        """Cell-centred node coordinates along axis a (0=x, 1=y, 2=z)."""
        N, L = self.n[a], self.L[a]
        return -L + (np.arange(N) + 0.5) * (2.0 * L / N)

    def axis_index(self, a):
        """Signed DFT index m for each position, in DFT order."""
        N = self.n[a]
        i = np.arange(N)
        return np.where(i < N // 2, i, i - N)

    def axis_k(self, a):
        """Wavenumbers k = pi m / L (true values, Nyquist included)."""
        return np.pi * self.axis_index(a) / self.L[a]

    def axis_k_odd(self, a):
        """Wavenumbers for odd factors: Nyquist entry set to zero."""
        k = self.axis_k(a).copy()
        k[self.n[a] // 2] = 0.0
        return k

    def mesh_nodes(self):
        """Node coordinate arrays X, Y, Z, each of shape (Nz, Ny, Nx)."""
        z, y, x = np.meshgrid(self.axis_nodes(2), self.axis_nodes(1), self.axis_nodes(0),
                              indexing="ij")
        return x, y, z

    def mesh_k(self, odd=False):
        """Wavenumber arrays KX, KY, KZ of shape (Nz, Ny, Nx)."""
        f = self.axis_k_odd if odd else self.axis_k
        kz, ky, kx = np.meshgrid(f(2), f(1), f(0), indexing="ij")
        return kx, ky, kz

    def k2(self):
        """|k|^2 with true wavenumbers."""
        kx, ky, kz = self.mesh_k(odd=False)
        return kx * kx + ky * ky + kz * kz

    def smoothing(self):
        """Gaussian smoothing multiplier S(k) = exp(-sigma^2 |k|^2 / 2)."""
        return np.exp(-0.5 * self.sigma ** 2 * self.k2())
