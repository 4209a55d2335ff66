"""Pins P2-P5 of the oracle's spectral operators.

P2  single Fourier modes: closed forms of C_s and Phi (signs, scales, axes,
    smoothing), on a non-cubic grid so a swapped axis fails
P3  operator identities: div C_s = 0, C_s Phi = S P, Phi C_s = S P on
    band-limited fields, mean(Phi[j]) = 0 (the k = 0 rule after Eq. 7)
P4  Eq. 6 == Eq. 7 on the grid: spectral Phi equals the direct circular
    convolution with its kernel built by the direct DFT
P5  Eq. 2 with G = 1/(4 pi |r|): spectral Phi of a Gaussian-magnetisation
    current approaches the exact free-space field as padding grows
"""
import numpy as np
import pytest
from scipy.special import erf

from oracle import brute, grid, operators
from paper_1803_01346_amd import workloads


def _mode_field(g, m, amp, fn):
    x, y, z = g.mesh_nodes()
    k = np.array([np.pi * m[0] / g.L[0], np.pi * m[1] / g.L[1], np.pi * m[2] / g.L[2]])
    ph = k[0] * x + k[1] * y + k[2] * z
    return k, np.stack([a * fn(ph) for a in amp]), ph


# grids of power-of-two and of 3 * 2^k lengths (the latter transformed by the
# direct DFT along each axis)
GRIDS = [(32, 16, 64), (48, 24, 96)]


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("m", [(3, 0, 0), (0, 2, 0), (0, 0, 5), (1, -2, 3)])
def test_curl_single_mode(m, n):
    g = grid.Grid(n, (2.0, 1.0, 3.0))
    a = np.array([0.3, -1.1, 0.7])
    k, h, ph = _mode_field(g, m, a, np.sin)
    got = operators.curl_s(h, g)
    s = np.exp(-0.5 * g.sigma ** 2 * np.dot(k, k))
    want = np.stack([c * np.cos(ph) for c in np.cross(k, a)]) * s     # (k x a) cos(k.r) S
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))


def test_curl_x_mode_matches_paper_orientation():
    # h = (0, 0, sin(k0 x)) -> curl h = (0, -k0 cos(k0 x), 0), times S(k0)
    g = grid.Grid((32, 8, 8), (2.0, 2.0, 2.0))
    x, _, _ = g.mesh_nodes()
    k0 = np.pi * 3 / 2.0
    h = np.stack([0 * x, 0 * x, np.sin(k0 * x)])
    got = operators.curl_s(h, g)
    s = np.exp(-0.5 * g.sigma ** 2 * k0 ** 2)
    assert np.max(np.abs(got[0])) < 1e-13 and np.max(np.abs(got[2])) < 1e-13
    assert np.max(np.abs(got[1] + k0 * np.cos(k0 * x) * s)) < 1e-12


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("m", [(3, 0, 0), (0, 2, 0), (0, 0, 5), (2, 1, -3)])
def test_phi_single_mode(m, n):
    # j = b cos(k.r) -> Phi[j] = -(k x b) sin(k.r) / |k|^2  (unsmoothed)
    g = grid.Grid(n, (2.0, 1.0, 3.0))
    b = np.array([1.0, 0.4, -0.6])
    k, j, ph = _mode_field(g, m, b, np.cos)
    got = operators.phi(j, g)
    want = -np.stack([c * np.sin(ph) for c in np.cross(k, b)]) / np.dot(k, k)
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, np.max(np.abs(want)))
    got_s = operators.phi(j, g, smooth=True)
    s = np.exp(-0.5 * g.sigma ** 2 * np.dot(k, k))
    assert np.max(np.abs(got_s - want * s)) < 1e-12 * max(1.0, np.max(np.abs(want)))


def test_phi_x_mode_closed_form():
    # j = (0, 0, J cos(k0 x)) -> Phi[j] = (0, J sin(k0 x) / k0, 0)
    g = grid.Grid((32, 8, 8), (2.0, 2.0, 2.0))
    x, _, _ = g.mesh_nodes()
    k0, J = np.pi * 3 / 2.0, 1.7
    j = np.stack([0 * x, 0 * x, J * np.cos(k0 * x)])
    got = operators.phi(j, g)
    assert np.max(np.abs(got[1] - J * np.sin(k0 * x) / k0)) < 1e-13
    assert np.max(np.abs(got[0])) < 1e-14 and np.max(np.abs(got[2])) < 1e-14


def _band_limited(n, L, seed):
    dh, _ = workloads.smooth_field(n, L, seed=seed, n_modes=10)
    return dh


def test_divergence_of_curl_is_zero_any_field():
    g = grid.Grid((16, 32, 8), (1.0, 2.0, 1.5))
    rng = np.random.default_rng(1)
    h = rng.normal(size=(3,) + g.shape)             # includes Nyquist content
    d = operators.div_s(operators.curl_s(h, g), g)
    j = operators.curl_s(h, g)
    assert np.max(np.abs(d)) < 1e-12 * np.max(np.abs(j)) * max(g.n) / min(g.L)


def test_curl_of_phi_is_smoothed_projection():
    g = grid.Grid((16, 32, 8), (1.0, 2.0, 1.5))
    j = _band_limited(g.n, g.L, 2)
    lhs = operators.curl_s(operators.phi(j, g), g)
    # S P j computed independently: smooth the projection by S in Fourier space
    Pj = operators.leray(j, g)
    from oracle import fft as F
    rhs_ = np.real(F.ifft3(F.fft3(Pj) * g.smoothing()))
    assert np.max(np.abs(lhs - rhs_)) < 1e-12 * np.max(np.abs(rhs_))


def test_phi_of_curl_is_smoothed_projection():
    g = grid.Grid((16, 32, 8), (1.0, 2.0, 1.5))
    a = _band_limited(g.n, g.L, 3)
    lhs = operators.phi(operators.curl_s(a, g), g)
    from oracle import fft as F
    rhs_ = np.real(F.ifft3(F.fft3(operators.leray(a, g)) * g.smoothing()))
    assert np.max(np.abs(lhs - rhs_)) < 1e-12 * np.max(np.abs(rhs_))


def test_phi_has_zero_mean():
    g = grid.Grid((16, 16, 16), (2.0, 2.0, 2.0))
    rng = np.random.default_rng(4)
    j = rng.normal(size=(3,) + g.shape) + 0.5       # nonzero mean on purpose
    p = operators.phi(j, g)
    assert np.max(np.abs(p.mean(axis=(1, 2, 3)))) < 1e-15 * np.max(np.abs(p)) * g.shape[0] ** 3


@pytest.mark.parametrize("n,L", [((8, 8, 8), (1.0, 1.0, 1.0)), ((8, 4, 16), (1.0, 0.7, 2.0))])
def test_phi_equals_direct_circular_sum(n, L):
    g = grid.Grid(n, L)
    rng = np.random.default_rng(5)
    j = rng.normal(size=(3,) + g.shape)
    K = brute.phi_kernel_direct(g)
    want = brute.circular_apply(K, j)
    got = operators.phi(j, g)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_curl_equals_direct_circular_sum():
    g = grid.Grid((8, 16, 4), (1.0, 2.0, 0.5))
    rng = np.random.default_rng(6)
    h = rng.normal(size=(3,) + g.shape)
    K = brute.curl_kernel_direct(g)
    want = brute.circular_apply(K, h)
    got = operators.curl_s(h, g)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def _gaussian_magnetisation_case(L, h, s=0.25):
    """j = curl(z f), f = exp(-r^2/(2 s^2)); exact field Phi_free[j] = z f + grad d_z u,
    u = Q erf(r / (sqrt2 s)) / (4 pi r), Q = (2 pi s^2)^(3/2)  (-lap u = f)."""
    n = int(round(2 * L / h))
    g = grid.Grid((n, n, n), (L, L, L))
    x, y, z = g.mesh_nodes()
    r = np.sqrt(x * x + y * y + z * z)
    f = np.exp(-r * r / (2 * s * s))
    j = np.stack([-y / s ** 2 * f, x / s ** 2 * f, 0 * f])
    Q = (2 * np.pi * s * s) ** 1.5
    A = erf(r / (np.sqrt(2) * s))
    A1 = np.sqrt(2 / np.pi) / s * np.exp(-r * r / (2 * s * s))
    A2 = -r / s ** 2 * A1
    c1 = (A2 * r * r - 3 * (A1 * r - A)) / (4 * np.pi * r ** 3)   # (g'' - g'/r)
    c2 = (A1 * r - A) / (4 * np.pi * r ** 3)                      # g'/r
    grad = [Q * c1 * xi * z / r ** 2 for xi in (x, y, z)]
    grad[2] = grad[2] + Q * c2
    exact = np.stack([grad[0], grad[1], grad[2] + f])
    return g, j, exact


def test_phi_approaches_free_space_field_with_padding():
    errs = []
    for L in (1.0, 2.0):
        g, j, exact = _gaussian_magnetisation_case(L, 1.0 / 16.0)
        got = operators.phi(j, g)
        # compare on the central region |x|,|y|,|z| < 0.75 common to both boxes
        x, y, z = g.mesh_nodes()
        core = (np.abs(x) < 0.75) & (np.abs(y) < 0.75) & (np.abs(z) < 0.75)
        errs.append(np.max(np.abs(got - exact)[:, core]) / np.max(np.abs(exact)))
    assert errs[1] < 0.25 * errs[0]          # periodic images fall off like 1/L^3
    assert errs[1] < 5e-3


def test_phi_matches_free_space_direct_sum_far_field():
    # nodes well outside the current: spectral Phi ~ direct Biot-Savart sum
    g, j, exact = _gaussian_magnetisation_case(1.5, 0.125, s=0.3)
    x, y, z = g.mesh_nodes()
    r = np.sqrt(x * x + y * y + z * z)
    tgt = (r > 1.0) & (r < 1.3)
    direct = brute.biot_savart_free(g, j * (r < 1.6), targets_mask=tgt)
    assert np.max(np.abs(direct - exact)[:, tgt]) < 0.015 * np.max(np.abs(exact[:, tgt]))
