"""Seeded synthetic workloads: the configurations' parameters, their shapes as
primitive lists, and smooth random vector fields.

This module holds inputs only.  It does no voxelization, no Fourier
transform and none of the method's operators: each consumer (the HIP
library, the CPU oracle used by tests) turns these specifications into
masks and fields by its own code.

Shapes are lists of primitives in units of the characteristic length l
(kind "box" | "cylinder" | "sphere", op "add" | "sub", center, size, axis):
  box       size = half-extents (ax, ay, az)
  cylinder  size = (radius, 0, half-height), axis = 0 | 1 | 2
  sphere    size = (radius, 0, 0)
"""
import math

import numpy as np


def prim(kind, op="add", center=(0.0, 0.0, 0.0), size=(0.0, 0.0, 0.0), axis=2):
    return dict(kind=kind, op=op, center=tuple(float(v) for v in center),
                size=tuple(float(v) for v in size), axis=int(axis))


def shape_cube(half_side=1.0):
    """Cube of side 2*half_side centred at the origin."""
    return [prim("box", "add", (0, 0, 0), (half_side,) * 3)]


def shape_cup(r_out=1.0, r_in=0.8, height=4.0, cap=0.2, axis=2):
    """Hollow cylinder closed at one end: bottom cap of thickness `cap`,
    open top; the hole reaches past the top face."""
    hh = 0.5 * height
    c = [0.0, 0.0, 0.0]
    c[axis] = cap                         # hole spans (-hh + cap, hh + cap)
    return [prim("cylinder", "add", (0, 0, 0), (r_out, 0.0, hh), axis),
            prim("cylinder", "sub", tuple(c), (r_in, 0.0, hh), axis)]


def shape_lens(radius=1.0, height=4.0 / 3.0, bore=0.2, slit=1.0 / 15.0):
    """Cylinder (axis z) with a coaxial bore and one radial slit along +x from
    the bore to the rim, both through the full height."""
    hh = 0.5 * height
    reach = 0.75 * radius                 # slit box spans x in (0, 1.5 R)
    return [prim("cylinder", "add", (0, 0, 0), (radius, 0.0, hh), 2),
            prim("cylinder", "sub", (0, 0, 0), (bore, 0.0, 2.0 * hh), 2),
            prim("box", "sub", (reach, 0.0, 0.0), (reach, 0.5 * slit, 2.0 * hh))]


def shape_cylinder(radius=1.0, height=2.0, axis=2):
    return [prim("cylinder", "add", (0, 0, 0), (radius, 0.0, 0.5 * height), axis)]


def shape_sphere(radius=1.0):
    return [prim("sphere", "add", (0, 0, 0), (radius, 0.0, 0.0))]


# --------------------------------------------------------------------------
# Configurations.  SI material and drive; geometry in units of l.
#   n           grid counts (Nx, Ny, Nz) of the padded FFT box
#   half_width  box half-widths in units of l
#   drive       kind ramp_hold | sine | pwl, direction, amplitude (T), ...
# rho_out: 20 for the shield-like and cube cases, 100 for the slit lens
# (the paper's own choices for its shield and lens).
# --------------------------------------------------------------------------

_S45 = math.sqrt(0.5)

CONFIGS = {
    # superconducting cube, side 1 cm, 16^3 voxels in a 32^3 box
    "cube32": dict(n=(32, 32, 32), l_m=5e-3, half_width=(2.0, 2.0, 2.0),
                   shapes=shape_cube(1.0), n_power=20.0, jc=1e8, e0=1e-4, rho_out=20.0,
                   drive=dict(kind="ramp_hold", direction=(0.0, 0.0, 1.0), amp_T=0.1,
                              t_ramp_s=1.0), t_end_s=2.0),
    # closed-end hollow cylinder R 10/8 mm, H 40 mm, cap 2 mm, 64^3 voxels in 128^3
    "cup128": dict(n=(128, 128, 128), l_m=10e-3, half_width=(4.0, 4.0, 4.0),
                   shapes=shape_cup(1.0, 0.8, 4.0, 0.2), n_power=100.0, jc=1e8, e0=1e-4,
                   rho_out=20.0,
                   drive=dict(kind="sine", direction=(_S45, 0.0, _S45), amp_T=0.05,
                              freq_hz=50.0), t_end_s=0.04),
    # the same shield on a coarser 64^3 box (32^3 voxels) for quick runs
    "cup64": dict(n=(64, 64, 64), l_m=10e-3, half_width=(4.0, 4.0, 4.0),
                  shapes=shape_cup(1.0, 0.8, 4.0, 0.2), n_power=100.0, jc=1e8, e0=1e-4,
                  rho_out=20.0,
                  drive=dict(kind="sine", direction=(_S45, 0.0, _S45), amp_T=0.05,
                             freq_hz=50.0), t_end_s=0.04),
    # bulk lens R 15 mm, H 20 mm, bore 3 mm, slit 1 mm, 128^3 voxels in 256^3
    "lens256": dict(n=(256, 256, 256), l_m=15e-3, half_width=(2.0, 2.0, 2.0),
                    shapes=shape_lens(1.0, 4.0 / 3.0, 0.2, 1.0 / 15.0), n_power=50.0,
                    jc=2e8, e0=1e-4, rho_out=100.0,
                    drive=dict(kind="ramp_hold", direction=(0.0, 0.0, 1.0), amp_T=1.0,
                               t_ramp_s=150.0), t_end_s=150.0),
}


MU0 = 4e-7 * np.pi


def shield_case(case="A", n_grid=128, tau=0.09, l_m=0.01, jc=1e8, e0=1e-4):
    """The shield run of Sec. 3 on a stand-in body (the paper's sizes come
    from a reference that is not available): a cup of outer radius 1, inner
    radius 0.8, height 2 and cap 0.2 (units of l, open end up) centred in the
    cube of side 3.2; n = 30, rho_out = 20; virgin start; the field grows
    along the axis and then across it (case A: (0, 0, t') then
    (t' - tau, 0, tau)) or in the opposite order (case B), t' up to 2 tau.
    Returns (cfg, t0_s, zone) with zone the shielded-zone primitive: a
    coaxial disk of radius 0.667 and thickness 0.143 whose middle plane is
    0.452 below the top of the cup."""
    t0 = MU0 * jc * l_m * l_m / e0
    bs = MU0 * jc * l_m                                  # tesla per unit of h'
    pts = {"A": [(0, 0, 0), (0, 0, tau), (tau, 0, tau)],
           "B": [(0, 0, 0), (tau, 0, 0), (tau, 0, tau)]}[case]
    cfg = dict(n=(n_grid,) * 3, l_m=l_m, half_width=(1.6, 1.6, 1.6),
               shapes=shape_cup(1.0, 0.8, 2.0, 0.2, axis=2), n_power=30.0, jc=jc, e0=e0, rho_out=20.0,
               drive=dict(kind="pwl", t_s=[0.0, tau * t0, 2 * tau * t0],
                          b_T=[[bs * v for v in p] for p in pts]))
    zone = prim("cylinder", "add", (0.0, 0.0, 1.0 - 0.452), (0.667, 0.0, 0.5 * 0.143), 2)
    return cfg, t0, zone


def config(name):
    return CONFIGS[name]


def batch_instances(count=64, seed=4, edges=(48, 64, 96, 128, 192)):
    """Independent instances of mixed size for batched runs: box edge drawn
    from `edges` (the body spans half of it: 24 to 96 voxels across), body
    (cube, solid cylinder or cup) with l = its half size, n ~ U[10, 100],
    log10 jc ~ U[7, 9], a ramp to U[0.01, 0.2] T along a random direction.
    Returns configuration dicts."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        edge = int(rng.choice(edges))
        kind = int(rng.integers(3))
        shapes = [shape_cube(1.0), shape_cylinder(1.0, 2.0), shape_cup(1.0, 0.8, 2.0, 0.2)][kind]
        d = rng.normal(size=3)
        out.append(dict(n=(edge, edge, edge), l_m=5e-3, half_width=(2.0, 2.0, 2.0), shapes=shapes,
                        n_power=float(rng.uniform(10.0, 100.0)), jc=float(10.0 ** rng.uniform(7.0, 9.0)),
                        e0=1e-4, rho_out=20.0,
                        drive=dict(kind="ramp_hold", direction=tuple(float(v) for v in d / np.linalg.norm(d)),
                                   amp_T=float(rng.uniform(0.01, 0.2)), t_ramp_s=1.0)))
    return out


# --------------------------------------------------------------------------
# Smooth random fields
# --------------------------------------------------------------------------

def smooth_field(n, half_width, seed=0, n_modes=12, max_index=None, j_target=1.05):
    """Random smooth periodic vector field on the node lattice and its exact
    continuum curl.

    dh(i) = sum_q a_q cos(2 pi (mx ix/Nx + my iy/Ny + mz iz/Nz) + p_q)
    with integer index vectors |m_a| <= max_index (default N_a/8, so there is
    no content near the Nyquist planes), Gaussian amplitude vectors a_q and
    uniform phases p_q.  The continuum curl, with k_a = pi m_a / L_a, is
    curl dh = -sum_q sin(...) (k_q x a_q); the field is scaled so that the
    largest node value of |curl dh| equals j_target.
    Returns (dh, curl_dh), each float64 of shape (3, Nz, Ny, Nx).
    """
    nx, ny, nz = (int(v) for v in n)
    rng = np.random.default_rng(seed)
    if max_index is None:
        max_index = (max(1, nx // 8), max(1, ny // 8), max(1, nz // 8))
    elif np.isscalar(max_index):
        max_index = (int(max_index),) * 3
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    dh = np.zeros((3, nz, ny, nx))
    cj = np.zeros((3, nz, ny, nx))
    for _ in range(n_modes):
        m = [int(rng.integers(-mi, mi + 1)) for mi in max_index]
        if m == [0, 0, 0]:
            m[0] = 1 if max_index[0] >= 1 else 0
        a = rng.normal(size=3)
        p = rng.uniform(0.0, 2.0 * np.pi)
        ph = 2.0 * np.pi * (m[0] * ix / nx + m[1] * iy / ny + m[2] * iz / nz) + p
        c, s = np.cos(ph), np.sin(ph)
        k = np.array([np.pi * m[0] / half_width[0], np.pi * m[1] / half_width[1],
                      np.pi * m[2] / half_width[2]])
        kxa = np.cross(k, a)
        for comp in range(3):
            dh[comp] += a[comp] * c
            cj[comp] -= kxa[comp] * s
    jmax = float(np.sqrt(np.max(np.sum(cj * cj, axis=0))))
    scale = j_target / jmax if jmax > 0 else 1.0
    return dh * scale, cj * scale


def synthetic_state_torch(cfg, seed=0, background=(0.0, 0.0, 0.0), n_modes=12, device="cuda"):
    """synthetic_state evaluated with torch on a device (the same modes,
    drawn from the same numpy generator; equal up to rounding): for large
    grids, where the host evaluation takes seconds."""
    import torch
    nx, ny, nz = (int(v) for v in cfg["n"])
    hw = cfg["half_width"]
    rng = np.random.default_rng(seed)
    max_index = (max(1, nx // 8), max(1, ny // 8), max(1, nz // 8))
    f64 = dict(dtype=torch.float64, device=device)
    ix = torch.arange(nx, **f64).view(1, 1, nx)
    iy = torch.arange(ny, **f64).view(1, ny, 1)
    iz = torch.arange(nz, **f64).view(nz, 1, 1)
    dh = torch.zeros((3, nz, ny, nx), **f64)
    cj = torch.zeros((3, nz, ny, nx), **f64)
    for _ in range(n_modes):
        m = [int(rng.integers(-mi, mi + 1)) for mi in max_index]
        if m == [0, 0, 0]:
            m[0] = 1
        a = rng.normal(size=3)
        p = rng.uniform(0.0, 2.0 * np.pi)
        ph = 2.0 * np.pi * (m[0] * ix / nx + m[1] * iy / ny + m[2] * iz / nz) + p
        c, sn = torch.cos(ph), torch.sin(ph)
        k = np.array([np.pi * m[0] / hw[0], np.pi * m[1] / hw[1], np.pi * m[2] / hw[2]])
        kxa = np.cross(k, a)
        for comp in range(3):
            dh[comp] += float(a[comp]) * c
            cj[comp] -= float(kxa[comp]) * sn
    jmax = float(torch.sqrt(torch.max(torch.sum(cj * cj, dim=0))))
    scale = 1.05 / jmax if jmax > 0 else 1.0
    b = torch.tensor(background, **f64).view(3, 1, 1, 1)
    return dh * scale + b


def synthetic_state(name_or_cfg, seed=0, background=(0.0, 0.0, 0.0), n=None, **kw):
    """h = uniform background + smooth_field(...) for a configuration."""
    cfg = CONFIGS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    n = cfg["n"] if n is None else n
    dh, _ = smooth_field(n, cfg["half_width"], seed=seed, **kw)
    b = np.asarray(background, dtype=np.float64).reshape(3, 1, 1, 1)
    return dh + b
