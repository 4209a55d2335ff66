"""Pins of the oracle's readouts, each against a fact fixed outside it.

moment          the moment of a magnetization current: for a localized,
                band-limited magnetization M and h = M, j = curl M and
                1/2 sum r x j dV = sum M dV (integration by parts), so the
                sign, the factor 1/2, the cell volume and the origin all
                show; the Gaussian smoothing (even) leaves it unchanged
magnetization   moment over the node volume of Omega
region_mean_abs a uniform field gives its magnitude; a one-node region the
                magnitude at that node
probe           trilinear interpolation reproduces node values at nodes and
                linear fields between them
stray_fraction  ||(1-chi) j|| / ||chi j|| against the closed-form current of
                a single Fourier mode (j = (k x a) cos(k.r) S(k))
"""
import numpy as np
import pytest

from oracle import grid, readouts


def _gauss_magnetization(g, m0, c, w):
    x, y, z = g.mesh_nodes()
    r2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    f = np.exp(-0.5 * r2 / w ** 2)
    return np.stack([m0[0] * f, m0[1] * f, m0[2] * f])


@pytest.mark.parametrize("n,L", [((48, 48, 48), (3.0, 3.0, 3.0)), ((48, 64, 48), (3.0, 4.0, 3.0))])
def test_moment_of_a_magnetization_current(n, L):
    # width 2.5 cells: the spectrum at the Nyquist wavenumber is e^-31 of its
    # peak, the box faces are 9 widths away (e^-40)
    g = grid.Grid(n, L)
    m0 = np.array([0.3, -0.7, 1.1])
    c = (0.1, -0.2, 0.15)                          # off-centre: the origin must not matter
    w = 2.5 * max(g.h)
    M = _gauss_magnetization(g, m0, c, w)
    want = M.reshape(3, -1).sum(axis=1) * g.cell_volume
    got = readouts.moment(g, np.ones(g.shape, np.uint8), M)
    assert np.max(np.abs(got - want)) <= 1e-11 * np.max(np.abs(want))
    # Omega covering the support: the Omega-only sum agrees to the smoothing spill
    chi = (np.sqrt(sum((a - b) ** 2 for a, b in zip(g.mesh_nodes(), c))) < 7 * w).astype(np.uint8)
    got_in = readouts.moment(g, chi, M, omega_only=True)
    assert np.max(np.abs(got_in - want)) <= 1e-6 * np.max(np.abs(want))
    vol = float(chi.sum()) * g.cell_volume
    assert np.allclose(readouts.magnetization(g, chi, M, omega_only=True), got_in / vol, rtol=1e-15)


def test_region_mean_abs():
    h = np.zeros((3, 4, 5, 6))
    h[0], h[1] = 3.0, 4.0
    assert readouts.region_mean_abs(h, np.ones((4, 5, 6), np.uint8)) == pytest.approx(5.0, rel=1e-15)
    rng = np.random.default_rng(2)
    h = rng.normal(size=(3, 4, 5, 6))
    one = np.zeros((4, 5, 6), np.uint8)
    one[2, 3, 1] = 1
    assert readouts.region_mean_abs(h, one) == pytest.approx(float(np.linalg.norm(h[:, 2, 3, 1])), rel=1e-15)
    assert readouts.region_mean_abs(h, np.zeros((4, 5, 6), np.uint8)) == 0.0


def test_probe_nodes_and_linear_fields():
    g = grid.Grid((8, 10, 12), (1.0, 1.25, 1.5))
    x, y, z = g.mesh_nodes()
    rng = np.random.default_rng(3)
    h = rng.normal(size=(3,) + g.shape)
    nodes = [(2, 3, 4), (0, 0, 0), (7, 9, 11)]
    pts = [(x[k, j, i], y[k, j, i], z[k, j, i]) for i, j, k in nodes]
    got = readouts.probe(g, h, pts)
    for p, (i, j, k) in enumerate(nodes):
        assert np.allclose(got[p], h[:, k, j, i], rtol=0, atol=1e-14)
    lin = np.stack([1.0 + 2.0 * x - y, 0.5 * z + x, 3.0 - z])
    q = np.array([[0.13, -0.41, 0.22], [-0.6, 0.7, -1.1], [0.0, 0.0, 0.0]])   # inside the node hull
    want = np.stack([1.0 + 2.0 * q[:, 0] - q[:, 1], 0.5 * q[:, 2] + q[:, 0], 3.0 - q[:, 2]], axis=1)
    assert np.allclose(readouts.probe(g, lin, q), want, rtol=0, atol=1e-13)


def test_stray_fraction_single_mode():
    g = grid.Grid((32, 16, 24), (2.0, 1.0, 1.5))
    x, y, z = g.mesh_nodes()
    m = (3, 1, -2)
    k = np.array([np.pi * m[0] / g.L[0], np.pi * m[1] / g.L[1], np.pi * m[2] / g.L[2]])
    a = np.array([0.4, -0.9, 0.5])
    ph = k[0] * x + k[1] * y + k[2] * z
    h = np.stack([c * np.sin(ph) for c in a])
    j = np.stack([c * np.cos(ph) for c in np.cross(k, a)]) * np.exp(-0.5 * g.sigma ** 2 * k @ k)
    chi = ((x > -0.7) & (x < 0.9) & (np.abs(y) < 0.6)).astype(np.uint8)
    w = chi.astype(float)
    want = np.sqrt(np.sum((j * (1 - w)) ** 2) / np.sum((j * w) ** 2))
    assert readouts.stray_fraction(g, chi, h) == pytest.approx(want, rel=1e-12)
    assert readouts.stray_fraction(g, np.ones(g.shape, np.uint8), h) == 0.0
