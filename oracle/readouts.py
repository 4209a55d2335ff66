"""Readouts of a state h (test infrastructure only).

  moment       m = 1/2 sum (r x j) dV with j = C_s h and r the node position
               from the box centre, summed over all nodes (default) or over
               Omega nodes only.  The all-node sum is unchanged by the
               Gaussian smoothing (an even kernel preserves first moments of
               a current with zero net flow), so it is the moment of the
               unsmoothed current; the Omega-only sum drops the part the
               smoothing spreads onto Omega_out.  (The paper reports field
               magnitudes; the moment is an added readout.)
  region_mean_abs   <|h|> over the nodes of a region mask (Sec. 3 compares
               the mean field magnitude in the shielded zone / lens central
               region with |h_e|)
  probe        trilinear interpolation of h at points (periodic wrap); on an
               axis between nodes this is the mean of the straddling nodes
  stray_fraction   ||(1-chi) j|| / ||chi j||: current left in Omega_out
"""
import numpy as np

from . import operators


def moment(grid, chi, h, omega_only=False):
    j = operators.curl_s(h, grid)
    x, y, z = grid.mesh_nodes()
    w = np.asarray(chi, dtype=np.float64) if omega_only else np.ones(grid.shape)
    jx, jy, jz = j[0] * w, j[1] * w, j[2] * w
    mx = 0.5 * np.sum(y * jz - z * jy) * grid.cell_volume
    my = 0.5 * np.sum(z * jx - x * jz) * grid.cell_volume
    mz = 0.5 * np.sum(x * jy - y * jx) * grid.cell_volume
    return np.array([mx, my, mz])


def magnetization(grid, chi, h, omega_only=False):
    """M = m / volume of Omega (node count times cell volume)."""
    vol = float(np.sum(chi)) * grid.cell_volume
    return moment(grid, chi, h, omega_only) / vol


def region_mean_abs(h, region):
    r = np.asarray(region) != 0
    mag = np.sqrt(h[0] ** 2 + h[1] ** 2 + h[2] ** 2)
    return float(np.mean(mag[r])) if np.any(r) else 0.0


def probe(grid, h, points):
    """h at arbitrary points by trilinear interpolation between nodes."""
    pts = np.atleast_2d(np.asarray(points, dtype=np.float64))
    out = np.zeros((pts.shape[0], 3))
    for p, xyz in enumerate(pts):
        idx, frac = [], []
        for a in range(3):
            s = (xyz[a] + grid.L[a]) / grid.h[a] - 0.5      # fractional node index
            i0 = int(np.floor(s))
            idx.append(i0)
            frac.append(s - i0)
        acc = np.zeros(3)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = ((frac[0] if dx else 1 - frac[0]) * (frac[1] if dy else 1 - frac[1])
                         * (frac[2] if dz else 1 - frac[2]))
                    ix = (idx[0] + dx) % grid.n[0]
                    iy = (idx[1] + dy) % grid.n[1]
                    iz = (idx[2] + dz) % grid.n[2]
                    acc += w * h[:, iz, iy, ix]
        out[p] = acc
    return out


def stray_fraction(grid, chi, h):
    j = operators.curl_s(h, grid)
    w = np.asarray(chi, dtype=np.float64)
    a = np.sqrt(np.sum((j * (1.0 - w)) ** 2))
    b = np.sqrt(np.sum((j * w) ** 2))
    return a / b if b > 0 else 0.0
