"""Pin P10: the Bogacki-Shampine 3(2) integrator."""
import numpy as np

from oracle import ode


def test_one_step_on_linear_ode_is_cubic_taylor():
    lam = -3.0
    for dt in (0.1, 0.01):
        z = lam * dt
        y1, k4, E = ode.bs23_step(lambda t, y: lam * y, 0.0, np.array([1.0]), dt, np.array([lam]))
        assert abs(y1[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


def test_third_order_convergence_fixed_steps():
    # y' = y cos t, y(0) = 1  ->  y = exp(sin t)
    f = lambda t, y: y * np.cos(t)
    errs = []
    for n in (20, 40, 80):
        y, st = ode.integrate(f, 0.0, 2.0, np.array([1.0]), fixed_steps=n)
        errs.append(abs(y[0] - np.exp(np.sin(2.0))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5


def test_error_estimate_is_third_order():
    f = lambda t, y: y * np.cos(t) + np.sin(3 * t)
    y0 = np.array([0.5])
    k1 = f(0.3, y0)
    es = []
    for dt in (0.04, 0.02, 0.01):
        _, _, E = ode.bs23_step(f, 0.3, y0, dt, k1)
        es.append(abs(E[0]))
    assert 6.5 < es[0] / es[1] < 9.5 and 6.5 < es[1] / es[2] < 9.5


def test_adaptive_meets_tolerance_and_hits_breakpoints():
    f = lambda t, y: np.where(t < 1.0, 1.0, -2.0 * y)       # kink at t = 1
    seen = []
    y, st = ode.integrate(f, 0.0, 3.0, np.array([0.0]), rtol=1e-6, atol=1e-9,
                          breakpoints=[1.0], observer=lambda t, y: seen.append(t))
    assert 1.0 in seen and seen[-1] == 3.0
    assert abs(y[0] - np.exp(-4.0)) < 1e-4
    assert st.accepted > 0 and all(e <= 1e-6 for e in st.err_hist)


def test_fsal_rhs_count():
    f = lambda t, y: -y
    y, st = ode.integrate(f, 0.0, 1.0, np.array([1.0]), fixed_steps=10)
    assert st.rhs_calls == 1 + 3 * 10
