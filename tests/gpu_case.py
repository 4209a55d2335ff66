"""Shared set-up for GPU parity tests: one configuration seen by both the
HIP library (through the C ABI) and the oracle (its own code)."""
import numpy as np

from oracle import geometry, grid, rhs, units
from paper_1803_01346_amd import scfft, workloads


def small_cfg(n, half_width, shapes, n_power=20.0, rho_out=20.0, drive=None, l_m=5e-3, jc=1e8):
    return dict(n=tuple(n), l_m=l_m, half_width=tuple(half_width), shapes=shapes,
                n_power=n_power, jc=jc, e0=1e-4, rho_out=rho_out,
                drive=drive or dict(kind="ramp_hold", direction=(0.0, 0.3, 1.0), amp_T=0.1,
                                    t_ramp_s=1.0))


def oracle_problem(cfg, **opt):
    g = grid.Grid(cfg["n"], cfg["half_width"])
    chi = geometry.voxelize(g, cfg["shapes"])
    u = units.Units(cfg["jc"], cfg["l_m"], cfg.get("e0", 1e-4))
    d = dict(cfg["drive"])
    dr = units.Drive(u, d.pop("kind"), **d)
    return rhs.Problem(g, chi, cfg["n_power"], cfg["rho_out"], dr, rhs.RhsOptions(**opt)), u


def sim(cfg, precision=scfft.F64, **opt):
    s = scfft.Simulation(cfg, precision=precision)
    if opt:
        scfft.scfft_set_rhs_opts(s.ctx, scfft.default_rhs_opts(**opt))
    return s


def state(cfg, seed=0, bg=(0.0, 0.02, 0.05), **kw):
    return workloads.synthetic_state(cfg, seed=seed, background=bg, **kw)


def to_dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def rel_max(x, r):
    return float(np.max(np.abs(x - r)) / max(np.max(np.abs(r)), 1e-300))


def rel_l2(x, r):
    return float(np.sqrt(np.sum((x - r) ** 2)) / max(np.sqrt(np.sum(r * r)), 1e-300))
