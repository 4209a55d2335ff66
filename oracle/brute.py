"""Brute-force sums that the spectral operators must reproduce
(test infrastructure only).

  phi_kernel_direct   K_Phi(r) = (1/Ntot) sum_k i [k_odd]_x / |k|^2 e^{i k.r}
                      evaluated with the direct DFT definition (no FFT);
                      [a]_x is the cross-product matrix, 0 at k = 0
  curl_kernel_direct  the same for C_s: S(k) i [k_odd]_x
  circular_apply      sum_q K(r_p - r_q) j(r_q), the direct O(N^2) sum over
                      node pairs on the periodic grid (Eq. 6 as a discrete
                      circular convolution)
  biot_savart_free    free-space Biot-Savart sum
                      h(r_p) = sum_{q != p} j(r_q) x (r_p - r_q) / (4 pi |r_p - r_q|^3) dV
                      (Eq. 2 with G = 1/(4 pi |r|)); a physical check only
"""
import numpy as np

from . import fft as _fft


def _cross_matrix(kx, ky, kz):
    """[k]_x such that [k]_x v = k x v; shape (3, 3, ...)."""
    z = np.zeros_like(kx)
    return np.array([[z, -kz, ky], [kz, z, -kx], [-ky, kx, z]])


def _kernel_from_symbol(grid, sym):
    """Real-space kernel K(r) = IDFT(sym) by the direct DFT, per matrix entry."""
    K = np.zeros((3, 3) + grid.shape)
    for a in range(3):
        for b in range(3):
            K[a, b] = np.real(_fft.dft3_direct(sym[a, b], inverse=True))
    return K


def phi_kernel_direct(grid, smooth=False):
    kx, ky, kz = grid.mesh_k(odd=True)
    k2 = grid.k2()
    inv = np.zeros_like(k2)
    inv[k2 != 0] = 1.0 / k2[k2 != 0]
    if smooth:
        inv = inv * grid.smoothing()
    sym = 1j * _cross_matrix(kx, ky, kz) * inv
    return _kernel_from_symbol(grid, sym)


def curl_kernel_direct(grid):
    kx, ky, kz = grid.mesh_k(odd=True)
    sym = 1j * _cross_matrix(kx, ky, kz) * grid.smoothing()
    return _kernel_from_symbol(grid, sym)


def circular_apply(K, v):
    """out[a](p) = sum_q sum_b K[a, b](p - q mod N) v[b](q): direct double sum."""
    _, _, nz, ny, nx = K.shape
    out = np.zeros_like(v, dtype=np.float64)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    iz, iy, ix = iz.ravel(), iy.ravel(), ix.ravel()
    vf = v.reshape(3, -1)
    for p in range(iz.size):
        dz = (iz[p] - iz) % nz
        dy = (iy[p] - iy) % ny
        dx = (ix[p] - ix) % nx
        Kp = K[:, :, dz, dy, dx]                    # (3, 3, nq)
        val = np.einsum("abq,bq->a", Kp, vf)
        out[:, iz[p], iy[p], ix[p]] = val
    return out


def biot_savart_free(grid, j, targets_mask=None):
    """Free-space Biot-Savart field of node currents j at the target nodes."""
    x, y, z = grid.mesh_nodes()
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    jf = j.reshape(3, -1).T
    src = np.any(jf != 0.0, axis=1)
    ps, js = pos[src], jf[src]
    if targets_mask is None:
        tgt = np.arange(pos.shape[0])
    else:
        tgt = np.flatnonzero(np.asarray(targets_mask).ravel())
    out = np.zeros((3, pos.shape[0]))
    for p in tgt:
        d = pos[p] - ps
        r2 = np.sum(d * d, axis=1)
        ok = r2 > 0
        w = 1.0 / (4.0 * np.pi * r2[ok] ** 1.5)
        out[:, p] = np.sum(np.cross(js[ok], d[ok]) * w[:, None], axis=0) * grid.cell_volume
    return out.reshape((3,) + grid.shape)
