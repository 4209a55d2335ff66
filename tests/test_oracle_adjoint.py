"""Pins of the oracle's reverse-mode derivatives (right-hand side with a fixed
iteration count and explicit warm start; fixed-step BS23).

* n = 1 (Ohm's law in Omega too) makes the right-hand side affine in
  (h, w, hedot): the adjoint identity <lam, df> + <mu, dw'> = <hbar, dh> +
  <wbar, dw> + <hedot_bar, dhedot> then holds to round-off for any finite
  increment, independent of finite-difference error.
* n = 20: central differences of the forward oracle (relative step 1e-6) for
  h, w, n, the kappa map and the drive vector, through one call and through
  a fixed-step integration.
"""
import numpy as np

from oracle import adjoint, geometry, grid, operators, rhs, units
from paper_1803_01346_amd import workloads


def _problem(npow=20.0, kappa=None, n=(8, 8, 8), fixed_iter=2, amp=0.1, direction=(0.0, 0.3, 1.0)):
    g = grid.Grid(n, (1.0, 1.0, 1.0))
    chi = geometry.voxelize(g, workloads.shape_cube(0.5))
    u = units.Units(1e8, 5e-3)
    d = units.Drive(u, "ramp_hold", direction, amp, 1.0)
    return rhs.Problem(g, chi, npow, 20.0, d, rhs.RhsOptions(fixed_iter=fixed_iter), kappa=kappa)


def _field(p, seed, scale=1.0):
    dh, _ = workloads.smooth_field(p.grid.n, p.grid.L, seed=seed, j_target=1.05, max_index=2)
    return scale * dh


def _state(p, seed):
    """A state whose smoothed current reaches 1.05 in Omega, so the power law
    is neither negligible nor huge."""
    dh = _field(p, seed)
    j = operators.curl_s(dh, p.grid)
    a = np.sqrt(np.sum(j * j, axis=0))[p.chi != 0]
    return dh * (1.05 / float(np.max(a)))


def _dot(a, b):
    return float(np.sum(a * b))


def _outside(p, v):
    return v * (1.0 - p.chi.astype(np.float64))


def test_affine_case_adjoint_identity():
    p = _problem(npow=1.0)
    t = 0.01
    h, v = _field(p, 1), _field(p, 2)
    w, dw = _outside(p, _field(p, 3)), _outside(p, _field(p, 4))
    lam, mu = _field(p, 5), _field(p, 6)
    for warm_used in (True, False):
        w0 = w if warm_used else None
        w1 = (w + dw) if warm_used else None
        f0, o0 = adjoint.rhs_forward(p, t, h, w0)
        f1, o1 = adjoint.rhs_forward(p, t, h + v, w1)
        lhs = _dot(lam, f1 - f0) + _dot(mu, o1 - o0)
        r = adjoint.rhs_vjp(p, t, h, warm_used, lam, mu)
        rhs_ = _dot(r["h_bar"], v) + (_dot(r["w_bar"], dw) if warm_used else 0.0)
        assert abs(lhs - rhs_) <= 1e-12 * max(abs(lhs), 1.0), (warm_used, lhs, rhs_)
    # hedot enters affinely through the exterior update (Eq. 5)
    q = _problem(npow=1.0, amp=0.13)
    f0, o0 = adjoint.rhs_forward(p, t, h, w)
    f1, o1 = adjoint.rhs_forward(q, t, h, w)
    dhe = np.asarray(q.drive.hedot(t)) - np.asarray(p.drive.hedot(t))
    r = adjoint.rhs_vjp(p, t, h, True, lam, mu)
    lhs = _dot(lam, f1 - f0) + _dot(mu, o1 - o0)
    assert abs(lhs - float(r["hedot_bar"] @ dhe)) <= 1e-12 * abs(lhs)


def _fd(fun, eps):
    return (fun(eps) - fun(-eps)) / (2.0 * eps)


def test_power_law_vjp_against_central_differences():
    kap = 1.0 + 0.1 * np.random.default_rng(7).normal(size=(8, 8, 8))
    p = _problem(npow=20.0, kappa=kap)
    t = 0.01
    h = _state(p, 11) + np.array([0.0, 0.0, 0.1]).reshape(3, 1, 1, 1)
    w = _outside(p, _field(p, 12, 0.3))
    lam, mu = _field(p, 13), _field(p, 14)
    r = adjoint.rhs_vjp(p, t, h, True, lam, mu)

    def J(hh=h, ww=w, prob=p):
        f, o = adjoint.rhs_forward(prob, t, hh, ww)
        return _dot(lam, f) + _dot(mu, o)

    v = _field(p, 15)
    s = 1e-6 * float(np.max(np.abs(h)))
    fd = _fd(lambda e: J(hh=h + e * v), s)
    assert abs(fd - _dot(r["h_bar"], v)) <= 1e-6 * abs(fd)
    dw = _outside(p, _field(p, 16))
    fd = _fd(lambda e: J(ww=w + e * dw), 1.0)      # affine in w: any step is exact
    assert abs(fd - _dot(r["w_bar"], dw)) <= 1e-10 * abs(fd)

    def Jn(e):
        q = _problem(npow=20.0 + e, kappa=kap)
        return J(prob=q)
    fd = _fd(Jn, 1e-6 * 20.0)
    assert abs(fd - r["n_bar"]) <= 1e-5 * abs(fd)

    dk = np.random.default_rng(8).normal(size=(8, 8, 8))

    def Jk(e):
        q = _problem(npow=20.0, kappa=kap + e * dk)
        return J(prob=q)
    fd = _fd(Jk, 1e-6)
    assert abs(fd - _dot(r["kappa_bar"], dk)) <= 1e-5 * abs(fd)


def test_integrator_adjoint_against_central_differences():
    p = _problem(npow=20.0)
    t0, t1, steps = 0.0, 2e-3, 3
    y0 = _state(p, 21) + np.array([0.0, 0.0, 0.05]).reshape(3, 1, 1, 1)
    ybar = _field(p, 22)
    yT, g = adjoint.integrate_adjoint(p, t0, t1, y0, steps, ybar)

    def L(yy=y0, prob=p):
        y, _ = adjoint.integrate_forward(prob, t0, t1, yy, steps)
        return _dot(ybar, y)

    assert abs(L() - _dot(ybar, yT)) == 0.0
    v = _field(p, 23)
    fd = _fd(lambda e: L(yy=y0 + e * v), 1e-6)
    assert abs(fd - _dot(g["y0_bar"], v)) <= 1e-6 * abs(fd)
    fd = _fd(lambda e: L(prob=_problem(npow=20.0 + e)), 2e-5)
    assert abs(fd - g["n_bar"]) <= 1e-5 * abs(fd)
    # drive vector p = amp * direction: scaling the amplitude by (1 + e) moves p by e p
    pvec = p.drive.dir * p.drive.amp
    fd = _fd(lambda e: L(prob=_problem(npow=20.0, amp=0.1 * (1.0 + e))), 1e-6)
    assert abs(fd - float(g["p_bar"] @ pvec)) <= 1e-6 * abs(fd)


def test_adjoint_of_zero_cotangent_is_zero():
    p = _problem()
    h = _field(p, 31)
    z = np.zeros_like(h)
    r = adjoint.rhs_vjp(p, 0.01, h, True, z, z)
    assert not np.any(r["h_bar"]) and not np.any(r["w_bar"]) and r["n_bar"] == 0.0
