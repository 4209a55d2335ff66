"""Pins P7-P9 of the oracle's right-hand side (Sec. 2, iteration of Eq. 5)."""
import numpy as np
import pytest

from oracle import geometry, grid, operators, rhs, units
from paper_1803_01346_amd import workloads


def _problem(n=(16, 16, 16), L=(2.0, 2.0, 2.0), shapes=None, npow=20.0, rho_out=20.0,
             direction=(0.0, 0.0, 1.0), **opt):
    g = grid.Grid(n, L)
    chi = geometry.voxelize(g, shapes if shapes is not None else workloads.shape_cube(1.0))
    u = units.Units(1e8, 5e-3)
    d = units.Drive(u, "ramp_hold", direction, 0.1, 1.0)
    return rhs.Problem(g, chi, npow, rho_out, d, rhs.RhsOptions(**opt))


def _state(p, seed=0, bg=(0.0, 0.0, 0.1)):
    dh, _ = workloads.smooth_field(p.grid.n, p.grid.L, seed=seed, j_target=1.05)
    return dh + np.asarray(bg).reshape(3, 1, 1, 1)


def test_rhs_is_odd_bitwise():
    # f(-h; -h_e) = -f(h; h_e) exactly: every step of the pipeline is odd
    p1 = _problem(fixed_iter=0)
    p2 = _problem(fixed_iter=0, direction=(0.0, 0.0, -1.0))
    h = _state(p1)
    a = rhs.rhs_eval(p1, 0.01, h)
    b = rhs.rhs_eval(p2, 0.01, -h)
    assert np.array_equal(b, -a)
    a2 = rhs.rhs_eval(p1, 0.02, h)             # warm start path too
    b2 = rhs.rhs_eval(p2, 0.02, -h)
    assert np.array_equal(b2, -a2)


def test_cube_axis_permutation_symmetry():
    # swapping x and z (grid axes and components) maps solutions to solutions
    pz = _problem(direction=(0.0, 0.0, 1.0), fixed_iter=4)
    px = _problem(direction=(1.0, 0.0, 0.0), fixed_iter=4)
    hz = _state(pz, bg=(0.0, 0.0, 0.1))

    def swap(v):
        return np.transpose(v[[2, 1, 0]], (0, 3, 2, 1))

    a = rhs.rhs_eval(pz, 0.01, hz)
    b = rhs.rhs_eval(px, 0.01, swap(hz))
    assert np.max(np.abs(swap(a) - b)) < 1e-11 * np.max(np.abs(a))


def test_iteration_contracts_and_converges():
    p = _problem(delta_it=1e-10, max_iter=60)
    h = _state(p)
    rhs.rhs_eval(p, 0.01, h)
    d = np.array(p.last_deltas)
    assert p.last_converged
    assert len(d) >= 3
    ratios = d[1:] / d[:-1]
    assert np.all(ratios < 0.9)                   # geometric decrease


def test_fixed_point_independent_of_warm_start():
    p = _problem(delta_it=1e-12, max_iter=200)
    h = _state(p)
    a = rhs.rhs_eval(p, 0.01, h)                 # Ohm-law start
    rng = np.random.default_rng(9)
    p.warm = rng.normal(size=a.shape)            # arbitrary warm start
    b = rhs.rhs_eval(p, 0.01, h)
    assert np.max(np.abs(a - b)) < 1e-8 * np.max(np.abs(a))


def test_stopping_rule_and_min_max_iter():
    p = _problem(delta_it=2e-5)
    h = _state(p)
    rhs.rhs_eval(p, 0.01, h)
    tol = 2e-5 * max(np.linalg.norm(p.drive.hedot(0.01)), 1.0)
    assert p.last_deltas[-1] < tol and all(x >= tol for x in p.last_deltas[:-1])
    q = _problem(delta_it=1e-30, max_iter=3)
    rhs.rhs_eval(q, 0.01, h)
    assert q.last_iters == 3 and not q.last_converged
    f = _problem(fixed_iter=2)
    rhs.rhs_eval(f, 0.01, h)
    assert f.last_iters == 2


def test_interior_rate_is_minus_curl_e():
    # inside Omega, hdot = -curl e with e from Eq. 1 (Eq. 3, fixed by the iteration)
    p = _problem(fixed_iter=3)
    h = _state(p)
    hd = rhs.rhs_eval(p, 0.01, h)
    from oracle import law
    j = operators.curl_s(h, p.grid)
    e = law.constitutive(j, p.chi, p.n, p.rho_out)
    want = -operators.curl_s(e, p.grid)
    m = p.chi == 1
    assert np.max(np.abs(hd[:, m] - want[:, m])) <= 1e-14 * np.max(np.abs(want))


def _far_stray(p, hd):
    jd = operators.curl_s(hd, p.grid)
    x, y, z = p.grid.mesh_nodes()
    dist = np.maximum(np.maximum(np.abs(x), np.abs(y)), np.abs(z)) - 1.0   # cube half-side 1
    far = dist > 4 * p.grid.sigma
    return np.sqrt(np.sum(jd[:, far] ** 2)), far


def test_exterior_current_suppressed_away_from_surface():
    # iteration (5) removes the current rate that the Ohm-law start leaves in
    # Omega_out; what remains beyond the smoothing layer is the gradient part of
    # the projection of the masked current, small and shrinking with iterations
    from oracle import law
    p1 = _problem(n=(32, 32, 32), fixed_iter=1)
    pc = _problem(n=(32, 32, 32), delta_it=1e-9, max_iter=300)
    h = _state(p1)
    a1, far = _far_stray(p1, rhs.rhs_eval(p1, 0.01, h))
    ac, _ = _far_stray(pc, rhs.rhs_eval(pc, 0.01, h))
    j = operators.curl_s(h, p1.grid)
    e = law.constitutive(j, p1.chi, p1.n, p1.rho_out)
    a0, _ = _far_stray(p1, -operators.curl_s(e, p1.grid))      # the Ohm-law start
    assert a1 < 0.02 * a0
    assert ac < 0.01 * a0 and ac < 0.7 * a1


def test_uniform_state_gives_applied_rate():
    # virgin state h = h_e: j = 0, e = 0, so hdot = 0 in Omega and the
    # exterior converges to the field of the shielding current rate
    p = _problem(delta_it=1e-10, max_iter=200)
    h = np.zeros((3,) + p.grid.shape)
    hd = rhs.rhs_eval(p, 0.0, h)
    assert np.all(hd[:, p.chi == 1] == 0.0)
    x, y, z = p.grid.mesh_nodes()
    far = np.maximum(np.maximum(np.abs(x), np.abs(y)), np.abs(z)) > 1.8
    hedot = p.drive.hedot(0.0)
    # far from the cube the rate is the applied rate plus a weak dipole field
    dev = np.abs(hd[2, far] - hedot[2]).mean() / hedot[2]
    assert dev < 0.3


def test_stopping_measure_hand_built():
    """The stopping measure of iteration (5) (Sec. 2, last paragraph) on hand-
    built iterates: the mean over Omega_out nodes of the Euclidean length of
    hdot^{i+1} - hdot^i.  A 4^3 grid with an 8-node Omega (n_out = 56); two
    Omega_out nodes move by (3, 4, 0) and (0, 0, -2), one Omega node by 100.
    Dividing by all nodes (7/64), the largest move (5 or 100), summing
    components (9/56), squares (29/56) or including Omega (107/56) all fail."""
    chi = np.zeros((4, 4, 4), dtype=np.uint8)
    chi[1:3, 1:3, 1:3] = 1
    old = np.random.default_rng(3).normal(size=(3, 4, 4, 4))
    new = old.copy()
    new[:, 0, 0, 0] += (3.0, 4.0, 0.0)
    new[:, 3, 2, 1] += (0.0, 0.0, -2.0)
    new[:, 1, 2, 1] += (100.0, 0.0, 0.0)
    assert abs(rhs.stopping_measure(new, old, chi) - 7.0 / 56.0) < 1e-14
    assert rhs.stopping_measure(new, old, np.ones_like(chi)) == 0.0     # no Omega_out


def test_first_delta_of_a_uniform_state_is_the_applied_rate():
    """With h uniform, j = C_s h vanishes to round-off, so e, hdot_in and the
    Ohm-law start vanish, and the first update of Eq. 5 sets hdot_out to the
    applied rate: d_0 = |dh_e/dt| (Euclidean, oblique drive) exactly as the
    stopping measure defines it."""
    p = _problem(fixed_iter=1, direction=(0.0, 0.6, 0.8))
    h = np.zeros((3,) + p.grid.shape) + np.array([0.0, 0.03, 0.04]).reshape(3, 1, 1, 1)
    rhs.rhs_eval(p, 0.25, h)
    rate = float(np.linalg.norm(p.drive.hedot(0.25)))
    assert abs(p.last_deltas[0] - rate) <= 1e-12 * rate


def test_recorded_deltas_are_the_stopping_measure_of_the_iterates():
    """Each recorded delta is the stopping measure of two consecutive
    iterates: rerunning with fixed_iter = i + 1 returns hdot^{i+1}."""
    h = _state(_problem())
    iterates = []
    for k in (1, 2, 3):
        q = _problem(fixed_iter=k)
        iterates.append(rhs.rhs_eval(q, 0.01, h))
    q = _problem(fixed_iter=3)
    rhs.rhs_eval(q, 0.01, h)
    for i in (1, 2):
        want = rhs.stopping_measure(iterates[i], iterates[i - 1], q.chi)
        assert abs(q.last_deltas[i] - want) <= 1e-12 * want
