"""Right-hand side of the method-of-lines system (test infrastructure only).

Follows Sec. 2 of the paper, in its order and notation, in the dimensionless
variables of Eq. 8 (mu0 = e0 = jc = 1):

  j = curl h                                   (Eq. 4, smoothed spectral curl)
  e = rho(|j|) j in Omega, rho_out j outside   (Eq. 1 and the Ohm-law start)
  hdot_in = -curl e restricted to Omega        (Eq. 3)
  hdot_out^0 = initial approximation in Omega_out
  iterate i = 0, 1, ...:
      jdot^i = curl hdot^i
      jdot_in^i = jdot^i in Omega, 0 in Omega_out
      hdot_out^{i+1} = hedot + Phi[jdot_in^i] restricted to Omega_out   (Eq. 5)
  until mean over Omega_out nodes of |hdot^{i+1} - hdot^i|
        < delta_it * max(|hedot|, 1)                     (stopping rule)

Readings (listed in the design notes):
  * the initial approximation is hdot_out from the most recent call
    ("from the previous time step"); on the first call, when none exists,
    it is the Ohm-law value -curl e on Omega_out;
  * min_iter (default 1) iterations always run; max_iter (default 200)
    stops with a not-converged flag; fixed_iter > 0 runs exactly that many;
  * |hedot| is the Euclidean norm at the evaluation time; the mean is over
    Omega_out nodes; an empty Omega_out counts as converged.
"""
import numpy as np

from . import law, operators


class RhsOptions:
    def __init__(self, delta_it=2e-5, min_iter=1, max_iter=200, fixed_iter=0,
                 smooth_phi=False):
        self.delta_it = float(delta_it)
        self.min_iter = int(min_iter)
        self.max_iter = int(max_iter)
        self.fixed_iter = int(fixed_iter)
        self.smooth_phi = bool(smooth_phi)


class Problem:
    """Everything rhs_eval needs besides the state: grid, mask, material,
    drive and options, plus the warm-start memory (hdot_out of the last call)."""

    def __init__(self, grid, chi, n_power, rho_out, drive, opts=None, kappa=None, field_law=None,
                 aniso=None):
        self.grid = grid
        self.chi = np.asarray(chi, dtype=np.uint8)
        self.n = float(n_power)
        self.rho_out = float(rho_out)
        self.drive = drive
        self.opts = opts if opts is not None else RhsOptions()
        self.kappa = kappa
        self.field_law = field_law  # (h_K, alpha): field-dependent critical density, or None
        self.aniso = aniso          # (a_x, a_y, a_z): anisotropic law, or None (isotropic)
        self.warm = None            # hdot on Omega_out from the most recent call
        self.last_iters = 0
        self.last_deltas = []
        self.last_converged = True


def stopping_measure(new, old, chi):
    """The quantity the stopping rule of iteration (5) tests (Sec. 2, last
    paragraph): the mean over the nodes of Omega_out (chi = 0) of the
    Euclidean length of hdot^{i+1} - hdot^i; 0 when Omega_out is empty."""
    out = np.asarray(chi) == 0
    n_out = int(np.sum(out))
    if n_out == 0:
        return 0.0
    diff = np.asarray(new) - np.asarray(old)
    mag = np.sqrt(diff[0] ** 2 + diff[1] ** 2 + diff[2] ** 2)
    return float(np.sum(mag[out]) / n_out)


def rhs_eval(prob, t, h):
    """hdot = f(t, h) for h of shape (3, Nz, Ny, Nx); updates prob.warm."""
    g = prob.grid
    inside = prob.chi.astype(np.float64)       # chi
    outside = 1.0 - inside                     # 1 - chi
    o = prob.opts

    j = operators.curl_s(h, g)                                   # Eq. 4
    e = law.constitutive(j, prob.chi, prob.n, prob.rho_out, prob.kappa, h, prob.field_law,
                         prob.aniso)                             # Eq. 1
    hdot_in = -operators.curl_s(e, g) * inside                   # Eq. 3 on Omega
    if prob.warm is None:
        hdot_out = -operators.curl_s(e, g) * outside             # Ohm-law start
    else:
        hdot_out = prob.warm * outside
    hdot = hdot_in + hdot_out

    hedot = np.asarray(prob.drive.hedot(t), dtype=np.float64).reshape(3, 1, 1, 1)
    tol = o.delta_it * max(float(np.sqrt(np.sum(hedot ** 2))), 1.0)
    deltas = []
    converged = False
    i = 0
    while True:
        jdot = operators.curl_s(hdot, g)                         # jdot^i = curl hdot^i
        jdot_in = jdot * inside                                  # zero in Omega_out
        new = hdot_in + outside * (hedot + operators.phi(jdot_in, g, o.smooth_phi))  # Eq. 5
        d = stopping_measure(new, hdot, prob.chi)
        deltas.append(d)
        hdot = new
        i += 1
        if o.fixed_iter > 0:
            if i >= o.fixed_iter:
                converged = True
                break
            continue
        if i >= o.min_iter and d < tol:
            converged = True
            break
        if i >= o.max_iter:
            converged = False
            break
    prob.warm = hdot * outside
    prob.last_iters = i
    prob.last_deltas = deltas
    prob.last_converged = converged
    return hdot
