"""Dimensionless scaling and applied-field drives (test infrastructure only).

Eq. 8: x' = x/l, t' = t/t0, e' = e/e0, j' = j/jc, h' = h/(jc l) with
t0 = mu0 jc l^2 / e0.  The applied field is given in tesla, B = mu0 h.
e0 = 1e-4 V/m (Sec. 2, after Eq. 1).

Drives (uniform applied field h_e(t), Sec. 2 problem statement):
  ramp_hold  B(t) = dir * amp * min(t / t_ramp, 1)
  sine       B(t) = dir * amp * sin(2 pi f t)
  pwl        B(t) piecewise linear through (t_k, B_k), constant outside
Each returns h_e'(t') and dh_e'/dt' in dimensionless units, and its kinks
(breakpoints, in t') so the integrator never steps over one.
"""
import numpy as np

MU0 = 4.0e-7 * np.pi
E0_DEFAULT = 1.0e-4


class Units:
    def __init__(self, jc, l, e0=E0_DEFAULT):
        self.jc = float(jc)
        self.l = float(l)
        self.e0 = float(e0)
        self.t0 = MU0 * self.jc * self.l ** 2 / self.e0
        self.h_scale = self.jc * self.l            # A/m per unit of h'

    def field_T_to_dimless(self, b):
        return np.asarray(b, dtype=np.float64) / MU0 / self.h_scale

    def field_dimless_to_T(self, h):
        return np.asarray(h, dtype=np.float64) * self.h_scale * MU0

    def time_s_to_dimless(self, t):
        return np.asarray(t, dtype=np.float64) / self.t0

    def length_m_to_dimless(self, x):
        return np.asarray(x, dtype=np.float64) / self.l

    def moment_dimless_to_Am2(self, m):
        # m = 1/2 int r x j dV:  r ~ l, j ~ jc, dV ~ l^3
        return np.asarray(m, dtype=np.float64) * self.jc * self.l ** 4


class Drive:
    """Uniform applied field; all methods take/return dimensionless t' and h'."""

    def __init__(self, units, kind, direction=(0.0, 0.0, 1.0), amp_T=0.0,
                 t_ramp_s=1.0, freq_hz=0.0, t_s=None, b_T=None):
        self.u = units
        self.kind = kind
        d = np.asarray(direction, dtype=np.float64)
        nrm = np.sqrt(np.sum(d * d))
        self.dir = d / nrm if nrm > 0 else d
        self.amp = float(units.field_T_to_dimless(amp_T))
        self.t_ramp = float(units.time_s_to_dimless(t_ramp_s))
        self.omega = 2.0 * np.pi * float(freq_hz) * units.t0   # rad per unit t'
        if kind == "pwl":
            self.tk = units.time_s_to_dimless(np.asarray(t_s, dtype=np.float64))
            self.bk = units.field_T_to_dimless(np.asarray(b_T, dtype=np.float64).reshape(-1, 3))
        elif kind not in ("ramp_hold", "sine"):
            raise ValueError("unknown drive kind %r" % kind)

    def he(self, t):
        if self.kind == "ramp_hold":
            return self.dir * self.amp * min(t / self.t_ramp, 1.0)
        if self.kind == "sine":
            return self.dir * self.amp * np.sin(self.omega * t)
        return self._pwl(t)[0]

    def hedot(self, t):
        """Time derivative; at a kink the right-hand derivative is returned."""
        if self.kind == "ramp_hold":
            return self.dir * (self.amp / self.t_ramp if t < self.t_ramp else 0.0)
        if self.kind == "sine":
            return self.dir * self.amp * self.omega * np.cos(self.omega * t)
        return self._pwl(t)[1]

    def _pwl(self, t):
        tk, bk = self.tk, self.bk
        if t < tk[0]:
            return bk[0].copy(), np.zeros(3)
        if t >= tk[-1]:
            return bk[-1].copy(), np.zeros(3)
        i = int(np.searchsorted(tk, t, side="right") - 1)
        dt = tk[i + 1] - tk[i]
        slope = (bk[i + 1] - bk[i]) / dt
        return bk[i] + slope * (t - tk[i]), slope

    def breakpoints(self):
        if self.kind == "ramp_hold":
            return [self.t_ramp]
        if self.kind == "pwl":
            return list(self.tk)
        return []
