"""The current-voltage relation (test infrastructure only).

Eq. 1: e = rho(|j|) j with rho(|j|) = (e0/jc) |j/jc|^(n-1).  In the
dimensionless variables of Eq. 8 (e' = e/e0, j' = j/jc) this is
    e' = |j'|^(n-1) j'.
With a local critical-density map kappa = jc(x)/jc_ref (an extension the
paper allows: "a different relation can also be employed"):
    e' = (|j'|/kappa)^(n-1) j'/kappa.
Outside the superconductor the fictitious Ohm law e = rho_out j is used
(the iteration paragraph of Sec. 2).  The oracle evaluates the plain
definition with a power; the GPU path uses a log form, and tests compare.
"""
import numpy as np


def power_law(j, n, kappa=None, aniso=None):
    """e' = (|j'|/kappa)^(n-1) j'/kappa, pointwise, e'(0) = 0.

    aniso = (a_x, a_y, a_z), all > 0: an anisotropic law (the paper allows
    other relations after Eq. 1 and fixes none; this form is user-chosen),
    the gradient in j' of the dissipation potential
        U(j') = kappa/(n+1) (|j'|_A/kappa)^(n+1),  |j'|_A^2 = sum_c a_c j'_c^2,
    that is e' = (|j'|_A/kappa)^(n-1) A j'/kappa with A = diag(a).  A = I is
    the isotropic law."""
    j = np.asarray(j, dtype=np.float64)
    w = np.ones(3) if aniso is None else np.asarray(aniso, dtype=np.float64)
    a = np.sqrt(w[0] * j[0] ** 2 + w[1] * j[1] ** 2 + w[2] * j[2] ** 2)
    if kappa is None:
        kappa = np.ones_like(a)
    r = a / kappa
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        rho = np.power(r, n - 1.0) / kappa
    rho = np.where(a > 0.0, rho, 0.0)
    return w.reshape((3,) + (1,) * (j.ndim - 1)) * j * rho


def field_kappa(kappa, h, field_law):
    """Field-dependent critical density (the e(j, h) relation that Sec. 2
    allows after Eq. 1; the paper fixes no form): a Kim-type decrease
    kappa_eff = kappa / (1 + |h| / h_K)^alpha with field_law = (h_K, alpha),
    h the local magnetic field, both dimensionless (Eq. 8)."""
    hk, alpha = field_law
    h = np.asarray(h, dtype=np.float64)
    mag = np.sqrt(h[0] ** 2 + h[1] ** 2 + h[2] ** 2)
    base = np.ones_like(mag) if kappa is None else np.asarray(kappa, dtype=np.float64)
    return base / np.power(1.0 + mag / hk, alpha)


def constitutive(j, chi, n, rho_out, kappa=None, h=None, field_law=None, aniso=None):
    """e = rho(|j|) j in the superconductor (chi = 1), rho_out j outside; with
    field_law the critical density depends on the local field h; with aniso
    the anisotropic law of power_law."""
    j = np.asarray(j, dtype=np.float64)
    inside = np.asarray(chi) != 0
    if field_law is not None:
        kappa = field_kappa(kappa, h, field_law)
    return np.where(inside, power_law(j, n, kappa, aniso), rho_out * j)
