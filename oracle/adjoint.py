"""Reverse-mode derivatives of the right-hand side and of fixed-step BS23
(test infrastructure only).

The paper integrates h forward; differentiating that discrete map is an
extension.  To make the map smooth it is taken with a fixed number K of
exterior iterations and with the warm start carried as an explicit state:

  f : (h, w) -> (hdot, w'),  w' = (1 - chi) hdot          (Sec. 2, Eq. 5 start)

with, in the notation of Sec. 2 (C = smoothed spectral curl, Eqs. 3-4;
Phi = Eq. 7; chi = mask of Omega):

  j = C h,   e = E(j) (Eq. 1 in Omega, rho_out j outside),   g = -C e
  hdot^0 = chi g + (1 - chi) w         (w absent on a first call: hdot^0 = g)
  hdot^{i+1} = chi g + (1 - chi) (hedot + Phi chi C hdot^i),  i < K   (Eq. 5)
  hdot = hdot^K

C and Phi have Hermitian symbols, so both are symmetric operators on real
periodic fields; the masks are diagonal; the Jacobian of E at a node of Omega
is rho(|j|) (I + (n - 1) jhat jhat^T), symmetric.  The adjoint therefore runs
the same operators in reverse order:

  l^K = lam + (1 - chi) mu,   l^i = C chi Phi (1 - chi) l^{i+1},   c = sum_{i>=1} l^i
  gbar = chi c + chi l^0 (warm start) or chi c + l^0 (first call)
  wbar = (1 - chi) l^0,  hedot_bar = sum over nodes of (1 - chi) c
  ebar = -C gbar,   jbar = dE/dj^T ebar,   hbar = C jbar
  nbar = sum_Omega ebar . e ln(|j|/kappa),   kappa_bar = -n ebar . e / kappa

Fixed-step BS23 (the tableau of the ode module) is differentiated step by
step, the warm start passing from each evaluation to the next in the order
k2, k3, k4 of every step (the first evaluation k1 of the run has none).
The applied field enters through hedot(t) = p f'(t) for drives of the form
h_e(t) = p f(t) (ramp-hold, sine); p_bar collects f'(t) hedot_bar over all
evaluations.
"""
import numpy as np

from . import law, ode, operators


def law_vjp(j, ebar, chi, n, rho_out, kappa=None):
    """jbar = (de/dj)^T ebar pointwise, and the parameter terms
    (nbar, kappa_bar per node) of Eq. 1."""
    inside = np.asarray(chi) != 0
    a = np.sqrt(j[0] ** 2 + j[1] ** 2 + j[2] ** 2)
    k = np.ones_like(a) if kappa is None else np.asarray(kappa, dtype=np.float64)
    pos = inside & (a > 0.0)
    safe = np.where(pos, a, 1.0)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        rho = np.where(pos, np.power(safe / k, n - 1.0) / k, 0.0)
    jhat = j / safe
    jhat_e = jhat[0] * ebar[0] + jhat[1] * ebar[1] + jhat[2] * ebar[2]
    jbar_in = rho * (ebar + (n - 1.0) * jhat * jhat_e)
    jbar = np.where(inside, jbar_in, rho_out * ebar)
    e = law.power_law(j, n, kappa)
    ebar_e = ebar[0] * e[0] + ebar[1] * e[1] + ebar[2] * e[2]
    nbar = float(np.sum(np.where(pos, ebar_e * np.log(safe / k), 0.0)))
    kappa_bar = np.where(pos, -n * ebar_e / k, 0.0)
    return jbar, nbar, kappa_bar


def rhs_forward(prob, t, h, warm):
    """(hdot, w') of one call with warm start `warm` (None: first call);
    prob.opts.fixed_iter must be > 0."""
    assert prob.opts.fixed_iter > 0
    from . import rhs
    prob.warm = None if warm is None else np.array(warm, copy=True)
    hdot = rhs.rhs_eval(prob, t, h)
    return hdot, prob.warm.copy()


def rhs_vjp(prob, t, h, warm_used, lam, mu=None):
    """Adjoint of one call: returns dict(h_bar, w_bar, n_bar, kappa_bar,
    hedot_bar) for the cotangent lam of hdot and mu of w'."""
    g = prob.grid
    K = prob.opts.fixed_iter
    assert K > 0
    assert prob.field_law is None, "reverse mode of the field-dependent law is not written"
    assert getattr(prob, "aniso", None) is None, "reverse mode of the anisotropic law is not written"
    inside = prob.chi.astype(np.float64)
    outside = 1.0 - inside
    # forward quantities the adjoint needs: j = C h (Eq. 4)
    j = operators.curl_s(h, g)
    # adjoint of the iteration (Eq. 5), last iterate first
    l = lam + (outside * mu if mu is not None else 0.0)
    c = l.copy()
    for i in range(K - 1, -1, -1):
        l = operators.curl_s(inside * operators.phi(outside * l, g, prob.opts.smooth_phi), g)
        if i > 0:
            c = c + l
    gbar = inside * c + (inside * l if warm_used else l)
    w_bar = outside * l
    hedot_bar = np.array([np.sum(outside * c[q]) for q in range(3)])
    # g = -C e (Eq. 3) and e = E(j) (Eq. 1)
    ebar = -operators.curl_s(gbar, g)
    jbar, nbar, kappa_bar = law_vjp(j, ebar, prob.chi, prob.n, prob.rho_out, prob.kappa)
    # j = C h (Eq. 4)
    h_bar = operators.curl_s(jbar, g)
    return dict(h_bar=h_bar, w_bar=w_bar, n_bar=nbar, kappa_bar=kappa_bar, hedot_bar=hedot_bar)


def drive_rate_factor(drive, t):
    """f'(t) for a drive h_e = p f(t): hedot(t) . p / |p|^2."""
    p = drive.dir * drive.amp
    pp = float(p @ p)
    return float(np.asarray(drive.hedot(t)) @ p) / pp if pp > 0.0 else 0.0


def integrate_forward(prob, t0, t1, y0, steps):
    """Fixed-step BS23 from y0 with a fresh warm start (as the GPU's adjoint
    integrator runs it); returns the final state and, per step, (t, dt, y,
    k1, k2) for the reverse sweep."""
    y = np.array(y0, dtype=np.float64, copy=True)
    dt = (t1 - t0) / steps
    warm = None
    k1, warm = rhs_forward(prob, t0, y, warm)
    tape = []
    t = float(t0)
    for s in range(steps):
        tn = t0 + (s + 1) * dt if s + 1 < steps else float(t1)
        h = tn - t
        k2, warm = rhs_forward(prob, t + ode.A21 * h, y + (ode.A21 * h) * k1, warm)
        k3, warm = rhs_forward(prob, t + ode.A32 * h, y + (ode.A32 * h) * k2, warm)
        y1 = y + h * (ode.B1 * k1 + ode.B2 * k2 + ode.B3 * k3)
        k4, warm = rhs_forward(prob, tn, y1, warm)
        tape.append((t, h, y, k1, k2))
        y, k1, t = y1, k4, tn
    return y, tape


def integrate_adjoint(prob, t0, t1, y0, steps, yT_bar):
    """Gradient of L(y_T) given yT_bar = dL/dy_T: returns (y_T, dict(y0_bar,
    n_bar, kappa_bar, p_bar))."""
    yT, tape = integrate_forward(prob, t0, t1, y0, steps)
    ybar = np.array(yT_bar, dtype=np.float64, copy=True)
    k1bar_next = np.zeros_like(ybar)     # cotangent of k1 of the next step (= k4 here)
    wbar = np.zeros_like(ybar)           # cotangent of the warm start leaving k4
    nbar = 0.0
    kbar_map = np.zeros(prob.grid.shape)
    pbar = np.zeros(3)

    def vjp(t, u, warm_used, lam, mu):
        nonlocal nbar, kbar_map, pbar
        r = rhs_vjp(prob, t, u, warm_used, lam, mu)
        nbar += r["n_bar"]
        kbar_map = kbar_map + r["kappa_bar"]
        pbar = pbar + drive_rate_factor(prob.drive, t) * r["hedot_bar"]
        return r["h_bar"], r["w_bar"]

    y_next = yT
    for (t, h, y, k1, k2) in reversed(tape):
        # k4 = f(t + h, y1; w3): its cotangent is that of the next k1
        u4bar, w3bar = vjp(t + h, y_next, True, k1bar_next, wbar)
        ybar = ybar + u4bar
        # y1 = y + h (B1 k1 + B2 k2 + B3 k3)
        k1bar = (ode.B1 * h) * ybar
        k2bar = (ode.B2 * h) * ybar
        k3bar = (ode.B3 * h) * ybar
        # k3 = f(t + A32 h, y + A32 h k2; w2)
        u3 = y + (ode.A32 * h) * k2
        u3bar, w2bar = vjp(t + ode.A32 * h, u3, True, k3bar, w3bar)
        ybar = ybar + u3bar
        k2bar = k2bar + (ode.A32 * h) * u3bar
        # k2 = f(t + A21 h, y + A21 h k1; w1)
        u2 = y + (ode.A21 * h) * k1
        u2bar, w1bar = vjp(t + ode.A21 * h, u2, True, k2bar, w2bar)
        ybar = ybar + u2bar
        k1bar = k1bar + (ode.A21 * h) * u2bar
        k1bar_next, wbar, y_next = k1bar, w1bar, y
    # the first evaluation k1 = f(t0, y0) had no warm start
    u1bar, _ = vjp(t0, y_next, False, k1bar_next, wbar)
    ybar = ybar + u1bar
    return yT, dict(y0_bar=ybar, n_bar=nbar, kappa_bar=kbar_map, p_bar=pbar)
