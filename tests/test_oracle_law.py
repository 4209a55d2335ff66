"""Pin P6: the power law of Eq. 1 in the dimensionless form of Eq. 8,
checked against closed forms that a dropped factor or a wrong exponent
would violate."""
import numpy as np
import pytest

from oracle import law


def _vec(a, d):
    d = np.asarray(d, float) / np.linalg.norm(d)
    return (a * d).reshape(3, 1)


@pytest.mark.parametrize("n", [1.0, 5.0, 20.0, 30.0, 100.0])
def test_critical_density_gives_e0(n):
    # |j| = jc  ->  e = e0 * j/|j|   (e' = j' when |j'| = 1)
    j = _vec(1.0, [0.3, -0.5, 0.8])
    e = law.power_law(j, n)
    assert np.allclose(e, j, rtol=1e-15, atol=0)


@pytest.mark.parametrize("n", [2.0, 20.0, 100.0])
@pytest.mark.parametrize("a", [1e-6, 0.3, 0.97, 1.0, 1.05, 2.0])
def test_magnitude_is_power_n(n, a):
    j = _vec(a, [1.0, 2.0, -2.0])
    e = law.power_law(j, n)
    assert np.isclose(np.linalg.norm(e), a ** n, rtol=1e-13)
    assert np.allclose(np.cross(e[:, 0], j[:, 0]), 0.0, atol=1e-14 * a ** n * a)  # e parallel to j


def test_zero_current_and_ohmic_case():
    assert np.all(law.power_law(np.zeros((3, 4)), 100.0) == 0.0)
    assert np.all(law.power_law(np.zeros((3, 4)), 1.0) == 0.0)
    rng = np.random.default_rng(0)
    j = rng.normal(size=(3, 10))
    assert np.allclose(law.power_law(j, 1.0), j, rtol=1e-15)       # n = 1: Ohm's law


def test_kappa_scaling():
    # (|j|/kappa)^(n-1) j / kappa: with j = kappa * u, e = |u|^(n-1) u
    rng = np.random.default_rng(1)
    u = rng.normal(size=(3, 20)) * 0.4
    kap = rng.uniform(0.5, 2.0, size=20)
    e = law.power_law(u * kap, 25.0, kappa=kap)
    assert np.allclose(e, law.power_law(u, 25.0), rtol=1e-13)


def test_constitutive_masks():
    rng = np.random.default_rng(2)
    j = rng.normal(size=(3, 2, 2, 2))
    chi = np.array([[[1, 0], [0, 1]], [[1, 1], [0, 0]]], dtype=np.uint8)
    e = law.constitutive(j, chi, 30.0, 20.0)
    assert np.allclose(e[:, chi == 0], 20.0 * j[:, chi == 0])
    assert np.allclose(e[:, chi == 1], law.power_law(j[:, chi == 1], 30.0))


def test_odd_and_isotropic():
    rng = np.random.default_rng(3)
    j = rng.normal(size=(3, 50))
    e = law.power_law(j, 30.0)
    assert np.array_equal(law.power_law(-j, 30.0), -e)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    assert np.allclose(law.power_law(q @ j, 30.0), q @ e, rtol=1e-12, atol=1e-14 * np.abs(e).max())


def test_field_dependent_critical_density():
    # e(j, h) allowed after Eq. 1: kappa_eff = kappa / (1 + |h|/h_K)^alpha
    rng = np.random.default_rng(3)
    j = rng.normal(size=(3, 4, 5, 6))
    chi = np.ones((4, 5, 6), dtype=np.uint8)
    h = rng.normal(size=(3, 4, 5, 6))
    kap = 1.0 + 0.1 * rng.normal(size=(4, 5, 6))
    base = law.constitutive(j, chi, 25.0, 20.0, kap)
    # alpha = 0, or a field far below h_K: the field-independent law
    assert np.array_equal(law.constitutive(j, chi, 25.0, 20.0, kap, h, (0.7, 0.0)), base)
    assert np.allclose(law.constitutive(j, chi, 25.0, 20.0, kap, h, (1e12, 1.0)), base, rtol=1e-9)
    # Kim model (alpha = 1): at |h| = h_K the critical density halves, so a
    # current of magnitude kappa/2 gives |e| = e0 (1 in Eq. 8 units)
    hk = 0.37
    hv = np.zeros((3, 4, 5, 6))
    hv[1] = hk
    u = j / np.sqrt(np.sum(j * j, axis=0))
    e = law.constitutive(u * (kap / 2.0), chi, 25.0, 20.0, kap, hv, (hk, 1.0))
    assert np.allclose(np.sqrt(np.sum(e * e, axis=0)), 1.0, rtol=1e-12)
    # outside the superconductor the field law does not enter
    chi0 = np.zeros((4, 5, 6), dtype=np.uint8)
    assert np.array_equal(law.constitutive(j, chi0, 25.0, 20.0, kap, h, (hk, 1.0)), 20.0 * j)


def _potential(j, n, kappa, a):
    # U(j) = kappa/(n+1) (|j|_A/kappa)^(n+1), |j|_A^2 = sum_c a_c j_c^2
    ja = np.sqrt(np.sum(np.asarray(a).reshape(3, 1) * j * j, axis=0))
    return kappa / (n + 1.0) * (ja / kappa) ** (n + 1.0)


@pytest.mark.parametrize("n", [1.0, 5.0, 30.0])
def test_anisotropic_law_is_the_gradient_of_its_potential(n):
    # e = grad_j U by central differences of U (a written-out potential, not
    # the law's formula): a dropped weight or a wrong exponent fails here
    rng = np.random.default_rng(11)
    a = (1.0, 0.4, 2.5)
    kap = 1.3
    j = rng.uniform(0.6, 1.2, size=(3, 8)) * rng.choice([-1.0, 1.0], size=(3, 8))
    e = law.power_law(j, n, np.full(8, kap), a)
    step = 1e-6
    for c in range(3):
        d = np.zeros((3, 1))
        d[c] = step
        fd = (_potential(j + d, n, kap, a) - _potential(j - d, n, kap, a)) / (2 * step)
        assert np.allclose(e[c], fd, rtol=1e-6, atol=1e-9)


def test_anisotropic_law_special_cases():
    rng = np.random.default_rng(12)
    j = rng.normal(size=(3, 40))
    kap = 1.0 + 0.2 * rng.random(40)
    # A = I: the isotropic law exactly
    assert np.array_equal(law.power_law(j, 25.0, kap, (1.0, 1.0, 1.0)), law.power_law(j, 25.0, kap))
    # A = lambda I: |j|_A = sqrt(lambda)|j|, so e scales by lambda^((n+1)/2)
    lam, n = 1.7, 9.0
    assert np.allclose(law.power_law(j, n, kap, (lam,) * 3), lam ** ((n + 1) / 2) * law.power_law(j, n, kap),
                       rtol=1e-12)
    # current along one axis: the one-dimensional law with critical density
    # kappa / sqrt(a_c), scaled by sqrt(a_c): e_c = a_c^((n+1)/2) (|j|/kappa)^(n-1) j/kappa
    a = (0.5, 2.0, 3.0)
    for c in range(3):
        jc = np.zeros((3, 40))
        jc[c] = j[c]
        e = law.power_law(jc, n, kap, a)
        want = a[c] ** ((n + 1) / 2) * (np.abs(j[c]) / kap) ** (n - 1) * j[c] / kap
        assert np.allclose(e[c], want, rtol=1e-12)
        assert np.all(e[[k for k in range(3) if k != c]] == 0.0)
    # odd, and dissipative: e . j = (|j|_A/kappa)^(n+1) kappa >= 0
    e = law.power_law(j, n, kap, a)
    assert np.array_equal(law.power_law(-j, n, kap, a), -e)
    ja = np.sqrt(np.sum(np.reshape(a, (3, 1)) * j * j, axis=0))
    assert np.allclose(np.sum(e * j, axis=0), (ja / kap) ** (n + 1) * kap, rtol=1e-12)
    # outside the superconductor the anisotropy does not enter
    chi0 = np.zeros(40, dtype=np.uint8)
    assert np.array_equal(law.constitutive(j, chi0, n, 20.0, kap, aniso=a), 20.0 * j)
