"""Method-of-lines time integration (test infrastructure only).

Sec. 2: the semi-discrete system for the node values of h is integrated with
Matlab's ode23 at relative tolerance 2e-4.  ode23 is the Bogacki-Shampine
3(2) pair (Bogacki & Shampine, Appl. Math. Lett. 2 (1989) 321-325) with the
first-same-as-last property.  The oracle implements that pair:

  k1 = f(t, y)                     (reused from the previous accepted step)
  k2 = f(t + dt/2,   y + dt/2 k1)
  k3 = f(t + 3dt/4,  y + 3dt/4 k2)
  y1 = y + dt (2/9 k1 + 1/3 k2 + 4/9 k3)
  k4 = f(t + dt, y1)
  E  = dt (-5/72 k1 + 1/12 k2 + 1/9 k3 - 1/8 k4)
  err = max_i |E_i| / max(|y_i|, |y1_i|, atol/rtol)    accept iff err <= rtol

Step-size control (a reading: the paper gives only RelTol):
  dt_new = dt * min(5, max(0.2, 0.8 (rtol/err)^(1/3))), not growing after a
  rejection; dt never crosses a breakpoint (drive kink) or the end time;
  after a breakpoint k1 is recomputed.  atol default 1e-6.
  Initial dt: 0.8 rtol^(1/3) / max_i(|f_i| / max(|y_i|, atol/rtol)), capped
  by dt_max and the interval.
Fixed-step mode: n equal steps, every step accepted.
"""
import numpy as np

A21 = 0.5
A32 = 0.75
B1, B2, B3 = 2.0 / 9.0, 1.0 / 3.0, 4.0 / 9.0
E1, E2, E3, E4 = -5.0 / 72.0, 1.0 / 12.0, 1.0 / 9.0, -1.0 / 8.0


class OdeStats:
    def __init__(self):
        self.accepted = 0
        self.rejected = 0
        self.rhs_calls = 0
        self.t_hist = []
        self.dt_hist = []
        self.err_hist = []


def err_norm(E, y, y1, rtol, atol):
    thr = atol / rtol
    scale = np.maximum(np.maximum(np.abs(y), np.abs(y1)), thr)
    return float(np.max(np.abs(E) / scale))


def bs23_step(f, t, y, dt, k1):
    """One Bogacki-Shampine step; returns y1, k4, E and the stage values."""
    k2 = f(t + A21 * dt, y + (A21 * dt) * k1)
    k3 = f(t + A32 * dt, y + (A32 * dt) * k2)
    y1 = y + dt * (B1 * k1 + B2 * k2 + B3 * k3)
    k4 = f(t + dt, y1)
    E = dt * (E1 * k1 + E2 * k2 + E3 * k3 + E4 * k4)
    return y1, k4, E


def integrate(f, t0, t1, y0, rtol=2e-4, atol=1e-6, dt0=0.0, dt_max=np.inf,
              breakpoints=(), fixed_steps=0, observer=None, max_steps=10 ** 7):
    """Integrate y' = f(t, y) from t0 to t1.  Returns (y, stats)."""
    st = OdeStats()
    y = np.array(y0, dtype=np.float64, copy=True)
    t = float(t0)
    stops = sorted(set([float(b) for b in breakpoints if t0 < b < t1] + [float(t1)]))

    def F(tt, yy):
        st.rhs_calls += 1
        return f(tt, yy)

    if fixed_steps > 0:
        dt = (t1 - t0) / fixed_steps
        k1 = F(t, y)
        for s in range(fixed_steps):
            tn = t0 + (s + 1) * dt if s + 1 < fixed_steps else float(t1)
            h = tn - t
            y1, k4, E = bs23_step(F, t, y, h, k1)
            st.err_hist.append(err_norm(E, y, y1, rtol, atol))
            st.t_hist.append(tn)
            st.dt_hist.append(h)
            st.accepted += 1
            y, t, k1 = y1, tn, k4
            if observer is not None:
                observer(t, y)
        return y, st

    k1 = F(t, y)
    thr = atol / rtol
    if dt0 > 0.0:
        dt = float(dt0)
    else:
        rate = float(np.max(np.abs(k1) / np.maximum(np.abs(y), thr)))
        dt = 0.8 * rtol ** (1.0 / 3.0) / rate if rate > 0.0 else (t1 - t0)
    dt = min(dt, dt_max, t1 - t0)
    si = 0
    rejected_last = False
    while t < t1 and st.accepted + st.rejected < max_steps:
        stop = stops[si]
        hit = False
        if t + dt >= stop or (stop - (t + dt)) < 1e-12 * max(abs(stop), 1.0):
            dt = stop - t
            hit = True
        y1, k4, E = bs23_step(F, t, y, dt, k1)
        err = err_norm(E, y, y1, rtol, atol)
        if not np.isfinite(err):
            err = np.inf
        if err <= rtol:
            t = stop if hit else t + dt
            y = y1
            k1 = k4
            st.accepted += 1
            st.t_hist.append(t)
            st.dt_hist.append(dt)
            st.err_hist.append(err)
            if observer is not None:
                observer(t, y)
            if hit:
                si += 1
                if si < len(stops) and stop < t1:
                    k1 = F(t, y)         # drive kink: no FSAL across it
            fac = 5.0 if err == 0.0 else min(5.0, max(0.2, 0.8 * (rtol / err) ** (1.0 / 3.0)))
            if rejected_last:
                fac = min(fac, 1.0)
            rejected_last = False
            dt = min(dt * fac, dt_max)
        else:
            st.rejected += 1
            fac = 0.2 if not np.isfinite(err) else max(0.2, 0.8 * (rtol / err) ** (1.0 / 3.0))
            dt = dt * min(fac, 0.5 if rejected_last else fac)
            rejected_last = True
            if dt < 1e-14 * max(abs(t), 1.0):
                raise FloatingPointError("step size underflow at t=%g" % t)
    return y, st
