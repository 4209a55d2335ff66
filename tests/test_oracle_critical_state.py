"""P11 on the oracle itself: the fully penetrated critical state of a cylinder
in an axial field (the Bean model at large n), reached by the oracle's own
right-hand side (Eqs. 1, 3, 4, 5, 7 with the stopping rule of Sec. 2) and
its own Bogacki-Shampine integrator, read out by its own moment.

Under a field ramp along the axis at rate hdot' (Eq. 8 units) a fully
penetrated body carries azimuthal current whose electric field is that of a
uniformly changing induction, |e| = hdot' rho / 2, so the power law (Eq. 1)
gives |j| = (hdot' rho / 2)^(1/n) and the magnetization is
M' = -(1/2) mean over the body of rho |j(rho)|: -R/3 for n -> inf (Bean),
and -(hdot' R / 2)^(1/n) R / (3 + 1/n) for the power law.

A start from the virgin state needs about 10^4 right-hand sides, which the
oracle cannot afford in a test, so the run starts from the analytic fully
penetrated field profile of the power law (the steady state does not depend
on the start) and integrates 0.04 time units, about ten relaxation times of
the critical-state current, with steps capped below the explicit stability
limit.  The body is a cylinder that spans the whole
periodic box along its axis (8 nodes, the cell a cube), i.e. the infinitely
long cylinder of the closed form.  The voxel surface carries less than the
critical current (staircase, smoothing width ~0.9 cell), so the moment
converges at first order in the cell size; two resolutions (8 and 12 cells
per radius) give the Richardson extrapolant, compared with the closed form
within 3 %.
"""
import numpy as np
import pytest

from oracle import geometry, grid, ode, readouts, rhs, units
from paper_1803_01346_amd import workloads

pytestmark = pytest.mark.slow

N_POW = 100.0
MU0 = 4e-7 * np.pi


def _run(cells_per_radius, t_span=0.04):
    n_xy = 4 * cells_per_radius                     # box [-2, 2)^2 across, radius 1
    cell = 4.0 / n_xy
    nz = 8
    lz = 0.5 * nz * cell
    g = grid.Grid((n_xy, n_xy, nz), (2.0, 2.0, lz))
    chi = geometry.voxelize(g, workloads.shape_cylinder(1.0, 4.0 * lz))
    l, jc, e0 = 0.01, 1e8, 1e-4
    u = units.Units(jc, l, e0)
    # h_e' = t' along z: amplitude 2 reached at t' = 2
    drive = units.Drive(u, "ramp_hold", (0.0, 0.0, 1.0), amp_T=2.0 * MU0 * jc * l,
                        t_ramp_s=2.0 * u.t0)
    prob = rhs.Problem(g, chi, N_POW, 20.0, drive, rhs.RhsOptions(delta_it=2e-5))
    x, y, _ = g.mesh_nodes()
    rho = np.sqrt(x * x + y * y)
    t0 = 1.5
    # h_z = h_e - int_rho^1 (s/2)^(1/n) ds inside, h_e outside
    q = 1.0 / N_POW
    inner = (N_POW / (N_POW + 1.0)) * (0.5 ** q - rho * (0.5 * rho) ** q)
    h = np.zeros((3,) + g.shape)
    h[2] = t0 - np.where(rho < 1.0, inner, 0.0)
    # steps capped below the explicit stability limit (~2.5 sigma^2 e / n): a
    # trial stage beyond it overflows the n = 100 law, and the warm start
    # would carry the overflow into every later call
    dt_max = 0.4 * g.sigma ** 2
    y1, st = ode.integrate(lambda t, v: rhs.rhs_eval(prob, t, v), t0, t0 + t_span, h,
                           dt0=0.1 * dt_max, dt_max=dt_max)
    m = readouts.moment(g, chi, y1)
    vol = float(chi.sum()) * g.cell_volume
    r = rho[chi != 0]
    want = -0.5 * float(np.mean(r * (0.5 * r) ** q))     # the voxel mask's own expectation
    return m[2] / vol, want, st


def test_oracle_cylinder_full_penetration():
    got8, want8, st8 = _run(8)
    got12, want12, st12 = _run(12)
    r8, r12 = got8 / want8, got12 / want12
    rich = 3.0 * r12 - 2.0 * r8                   # first order in the cell size: h = 1/8, 1/12
    bean = -(0.5 ** (1.0 / N_POW)) / (3.0 + 1.0 / N_POW)
    print("oracle cylinder: M' %.5f / %.5f (8 cells), %.5f / %.5f (12 cells); ratios %.4f %.4f, "
          "extrapolated %.4f; closed form %.5f; steps %d, %d"
          % (got8, want8, got12, want12, r8, r12, rich, bean, st8.accepted, st12.accepted))
    assert got8 < 0.0 and got12 < 0.0             # diamagnetic under an increasing field
    assert abs(r12 - 1.0) < abs(r8 - 1.0)         # the deficit shrinks with refinement
    assert abs(rich - 1.0) < 0.03
    # the mask's expectation is the closed form of the continuum cylinder up to voxelization
    assert abs(want12 / bean - 1.0) < 0.03
