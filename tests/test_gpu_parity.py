"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  FP64 path: operators <= 1e-12, right-hand side and
trajectories <= 1e-10 (relative to the largest reference value); FP32 path
<= 1e-4 relative L2."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import operators, readouts, rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUBE32 = workloads.config("cube32")
NONCUBIC = small_cfg((16, 32, 64), (1.5, 2.0, 3.0), workloads.shape_cup(1.0, 0.6, 3.0, 0.4, axis=1))
TINY = small_cfg((8, 8, 8), (1.0, 1.0, 1.0), workloads.shape_cube(0.5))
FLAT = small_cfg((64, 16, 8), (4.0, 1.0, 1.0), workloads.shape_cylinder(0.6, 1.2, axis=0))
CUP64 = workloads.config("cup64")
SQZ = small_cfg((32, 32, 16), (2.0, 2.0, 1.0), workloads.shape_cylinder(0.8, 1.2))


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("fuse", [2, 0])
@pytest.mark.parametrize("cfg", [TINY, NONCUBIC, FLAT, CUBE32, CUP64, SQZ],
                         ids=["8", "16x32x64", "64x16x8", "32", "64", "32x32x16"])
def test_curl_and_phi_fp64(cfg, fuse):
    s = sim(cfg, fuse_xy=fuse)
    g, _ = oracle_problem(cfg)
    rng = np.random.default_rng(1)
    v = rng.normal(size=s.field_shape)               # full-band input, Nyquist included
    dv = to_dev(torch, v, torch.float64)
    out = s.empty_field()
    scfft.scfft_curl(s.ctx, dv, out)
    torch.cuda.synchronize()
    want = operators.curl_s(v, g.grid)
    assert rel_max(_np(out), want) < 1e-12
    scfft.scfft_phi(s.ctx, dv, out)
    torch.cuda.synchronize()
    want = operators.phi(v, g.grid)
    assert rel_max(_np(out), want) < 1e-12


@pytest.fixture(scope="module")
def curl_phi_128():
    """Full-band random input (Nyquist planes included) on the 128^3 box and
    the oracle's C_s and Phi (Eq. 7, k = 0 rule) of it."""
    cfg = workloads.config("cup128")
    g, _ = oracle_problem(cfg)
    v = np.random.default_rng(11).normal(size=(3, 128, 128, 128))
    return cfg, v, operators.curl_s(v, g.grid), operators.phi(v, g.grid)


@pytest.mark.parametrize("fuse", [2, 0])
def test_curl_and_phi_fp64_128(fuse, curl_phi_128):
    cfg, v, want_curl, want_phi = curl_phi_128
    s = sim(cfg, fuse_xy=fuse)
    dv = to_dev(torch, v, torch.float64)
    out = s.empty_field()
    scfft.scfft_curl(s.ctx, dv, out)
    torch.cuda.synchronize()
    assert rel_max(_np(out), want_curl) < 1e-12
    scfft.scfft_phi(s.ctx, dv, out)
    torch.cuda.synchronize()
    assert rel_max(_np(out), want_phi) < 1e-12


# The headline workload: the shield on the 128^3 box (n = 100, rho_out = 20),
# 3 exterior iterations, the seeded critical-state state on the applied field
# of the 50 Hz drive at its peak; a first call (Ohm-law start of Eq. 5) and a
# second call that starts from the first call's exterior rate (Sec. 2).
T128 = (0.005, 0.00501)


@pytest.fixture(scope="module")
def cup128_rhs():
    cfg = workloads.config("cup128")
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=0, bg=tuple(prob.drive.he(T128[0] / u.t0)))
    want = [orhs.rhs_eval(prob, t_s / u.t0, h) for t_s in T128]
    return cfg, h, want


@pytest.mark.parametrize("fuse", [0, 2], ids=["rowcol", "plane"])
def test_rhs_fixed_iter_fp64_128_all_nodes(fuse, cup128_rhs):
    """Every node and component of the 128^3 right-hand side against the
    oracle (FP64 <= 1e-10 relative max), first and warm-started call, with
    the schedule the bench times (row/column passes, pruned to Omega's box)
    and with the fused plane passes."""
    cfg, h, want = cup128_rhs
    s = sim(cfg, fixed_iter=3, fuse_xy=fuse)
    dh = to_dev(torch, h, torch.float64)
    for t_s, w in zip(T128, want):
        out, _ = s.rhs_eval(t_s, dh)
        torch.cuda.synchronize()
        err = rel_max(_np(out), w)
        print("128^3 FP64 fuse_xy=%d t=%g: rel max %.2e" % (fuse, t_s, err))
        assert err < 1e-10, t_s


def test_rhs_fixed_iter_fp32_128_all_nodes(cup128_rhs):
    """The FP32 bulk path on the same workload and schedule against the FP64
    oracle: <= 1e-4 relative L2 over all nodes, first and warm-started call."""
    cfg, h, want = cup128_rhs
    s = sim(cfg, precision=scfft.F32, fixed_iter=3)
    dh = to_dev(torch, h, torch.float32)
    for t_s, w in zip(T128, want):
        out, _ = s.rhs_eval(t_s, dh)
        torch.cuda.synchronize()
        got = _np(out)
        print("128^3 FP32 t=%g: rel L2 %.2e, rel max %.2e" % (t_s, rel_l2(got, w), rel_max(got, w)))
        assert rel_l2(got, w) < 1e-4, t_s


@pytest.mark.parametrize("fuse", [2, 0])
@pytest.mark.parametrize("cfg", [TINY, NONCUBIC, CUBE32, CUP64, SQZ], ids=["8", "16x32x64", "32", "64", "32x32x16"])
def test_rhs_fixed_iter_fp64(cfg, fuse):
    s = sim(cfg, fixed_iter=3, fuse_xy=fuse)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=2)
    dh = to_dev(torch, h, torch.float64)
    for t_s in (0.25, 0.3):                            # second call uses the warm start
        out, st = s.rhs_eval(t_s, dh)
        torch.cuda.synchronize()
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        assert rel_max(_np(out), want) < 1e-10, t_s


@pytest.mark.parametrize("cfg", [NONCUBIC, CUBE32], ids=["16x32x64", "32"])
def test_rhs_adaptive_fp64(cfg):
    s = sim(cfg, delta_it=2e-5)
    prob, u = oracle_problem(cfg, delta_it=2e-5)
    h = state(cfg, seed=4)
    dh = to_dev(torch, h, torch.float64)
    for t_s in (0.2, 0.21, 0.22):
        stats = scfft.RhsStats()
        out, rc = s.rhs_eval(t_s, dh, stats=stats)
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        assert stats.iters == prob.last_iters
        assert abs(stats.last_delta - prob.last_deltas[-1]) <= 1e-9 * prob.last_deltas[-1]
        assert rel_max(_np(out), want) < 1e-10


@pytest.mark.parametrize("fuse", [2, 0])
def test_rhs_fp32_within_1e4(fuse):
    cfg = CUP64
    s = sim(cfg, precision=scfft.F32, fixed_iter=3, fuse_xy=fuse)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=5)
    out, _ = s.rhs_eval(0.004, to_dev(torch, h, torch.float32))
    torch.cuda.synchronize()
    want = orhs.rhs_eval(prob, 0.004 / u.t0, h)
    assert rel_l2(_np(out), want) < 1e-4


def test_rhs_is_odd_bitwise_on_gpu():
    cfg = CUP64
    s1 = sim(cfg, fixed_iter=3)
    cfg2 = dict(cfg, drive=dict(cfg["drive"], direction=tuple(-v for v in cfg["drive"]["direction"])))
    s2 = sim(cfg2, fixed_iter=3)
    h = to_dev(torch, state(cfg, seed=6), torch.float64)
    a, _ = s1.rhs_eval(0.003, h)
    b, _ = s2.rhs_eval(0.003, -h)
    torch.cuda.synchronize()
    assert torch.equal(b, -a)


def test_readouts_fp64():
    cfg = CUBE32
    s = sim(cfg)
    prob, u = oracle_problem(cfg)
    # a localized field (Gaussian window) so the moment is far above round-off
    x, y, z = prob.grid.mesh_nodes()
    h = state(cfg, seed=7) * np.exp(-(x * x + y * y + z * z) / 0.8)
    dh = to_dev(torch, h, torch.float64)
    for omega_only in (0, 1):
        m = scfft.scfft_moment(s.ctx, dh, omega_only)
        mo = readouts.moment(prob.grid, prob.chi, h, omega_only=bool(omega_only))
        mo_si = u.moment_dimless_to_Am2(mo)
        assert np.allclose(m, mo_si, rtol=1e-10, atol=1e-12 * np.max(np.abs(mo_si)))
    region = to_dev(torch, prob.chi, torch.uint8)
    b = scfft.scfft_region_mean_abs_b(s.ctx, dh, region)
    bo = u.field_dimless_to_T(readouts.region_mean_abs(h, prob.chi))
    assert abs(b - bo) <= 1e-12 * bo
    pts = np.array([[0.0, 0.0, 0.0], [1e-3, -2e-3, 3e-3], [0.009, 0.0, -0.0095]])
    pb = scfft.scfft_probe_b(s.ctx, dh, pts)
    po = u.field_dimless_to_T(readouts.probe(prob.grid, h, pts / cfg["l_m"]))
    assert np.allclose(pb, po, rtol=1e-12, atol=1e-15)


def test_init_state_and_virgin_rhs():
    cfg = CUBE32
    s = sim(cfg, fixed_iter=4)
    prob, u = oracle_problem(cfg, fixed_iter=4)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.5, h)
    he = prob.drive.he(0.5 / u.t0)
    assert np.allclose(_np(h), np.broadcast_to(he.reshape(3, 1, 1, 1), h.shape), rtol=1e-15)
    out, _ = s.rhs_eval(0.5, h)
    want = orhs.rhs_eval(prob, 0.5 / u.t0, _np(h))
    assert rel_max(_np(out), want) < 1e-10


@pytest.mark.parametrize("fuse", [2, 0])
def test_integrate_fixed_steps_fp64(fuse):
    """Stage arguments y + c k formed inside the first pass (plane pass or
    row pass) and the state kept in the workspace give the oracle's BS23."""
    cfg = dict(CUBE32, n_power=20.0)
    s = sim(cfg, fixed_iter=2, fuse_xy=fuse)
    prob, u = oracle_problem(cfg, fixed_iter=2)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    o = scfft.default_ode_opts(fixed_steps=6)
    st = scfft.OdeStats()
    ms = []
    scfft.scfft_integrate(s.ctx, 0.0, 0.02, h, o, observer=lambda u_, t, p: ms.append(t) or 0, stats=st)
    torch.cuda.synchronize()
    from oracle import ode
    f = lambda t, y: orhs.rhs_eval(prob, t, y)
    y, so = ode.integrate(f, 0.0, 0.02 / u.t0, np.zeros((3,) + prob.grid.shape), fixed_steps=6)
    assert st.accepted == 6 and st.rhs_calls == so.rhs_calls and len(ms) == 6
    assert rel_max(_np(h), y) < 1e-10


@pytest.mark.parametrize("prec,fuse", [(scfft.F64, 0), (scfft.F64, 2), (scfft.F32, 1)])
def test_step_moment_in_observer(prec, fuse):
    """The moment the power-law pass records for each accepted state equals the
    stand-alone readout of the state the observer sees, and the oracle's
    moment of the final state (Sec. 2 readout)."""
    cfg = dict(CUBE32, n_power=20.0)
    s = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=fuse)
    prob, u = oracle_problem(cfg, fixed_iter=2)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    # a localized field (Gaussian window) so the moment is far above round-off
    x, y, z = prob.grid.mesh_nodes()
    h = to_dev(torch, state(cfg, seed=5) * np.exp(-(x * x + y * y + z * z) / 0.8), dt)
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_step_moment(s.ctx)
    got = []

    def obs(_u, t, p):
        got.append((scfft.scfft_step_moment(s.ctx, 0), scfft.scfft_step_moment(s.ctx, 1),
                    scfft.scfft_moment(s.ctx, p, 0), scfft.scfft_moment(s.ctx, p, 1)))
        return 0

    o = scfft.default_ode_opts(fixed_steps=3)
    scfft.scfft_integrate(s.ctx, 0.0, 0.01, h, o, observer=obs)
    assert len(got) == 3
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    for m_all, m_in, r_all, r_in in got:
        assert np.max(np.abs(m_all - r_all)) <= tol * np.max(np.abs(r_all))
        assert np.max(np.abs(m_in - r_in)) <= tol * np.max(np.abs(r_in))
    # the last accepted state is h after the call: the oracle's moment of it
    hn = _np(h).astype(np.float64)
    want_all = u.moment_dimless_to_Am2(readouts.moment(prob.grid, prob.chi, hn))
    want_in = u.moment_dimless_to_Am2(readouts.moment(prob.grid, prob.chi, hn, omega_only=True))
    otol = 1e-10 if prec == scfft.F64 else 1e-4
    assert np.max(np.abs(got[-1][0] - want_all)) <= otol * np.max(np.abs(want_all))
    assert np.max(np.abs(got[-1][1] - want_in)) <= otol * np.max(np.abs(want_in))
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_step_moment(s.ctx)


def test_integrate_adaptive_fp64_agrees_with_oracle():
    cfg = small_cfg((16, 16, 16), (2.0, 2.0, 2.0), workloads.shape_cube(1.0), n_power=20.0,
                    drive=dict(kind="ramp_hold", direction=(0, 0, 1), amp_T=0.1, t_ramp_s=1.0))
    s = sim(cfg)
    prob, u = oracle_problem(cfg)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    o = scfft.default_ode_opts()
    st = scfft.OdeStats()
    scfft.scfft_integrate(s.ctx, 0.0, 1.5, h, o, stats=st)
    from oracle import ode
    f = lambda t, y: orhs.rhs_eval(prob, t, y)
    y, so = ode.integrate(f, 0.0, 1.5 / u.t0, np.zeros((3,) + prob.grid.shape),
                          breakpoints=prob.drive.breakpoints())
    # the two runs take the same decisions (their arithmetic agrees far below
    # the controller's margins), so the same steps and states
    assert (st.accepted, st.rejected, st.rhs_calls) == (so.accepted, so.rejected, so.rhs_calls)
    assert rel_max(_np(h), y) < 1e-10


def test_integrate_adaptive_shield_fp64_agrees_with_oracle():
    """The shield stand-in at 32^3 (n = 30, rho_out = 20, a transverse field
    ramp, the paper's stopping rule and step control) integrated adaptively
    on the GPU and by the oracle: the same accepted and rejected steps and
    the same state to 1e-10."""
    cfg, t0, _ = workloads.shield_case("B", 32)
    s = sim(cfg)
    prob, u = oracle_problem(cfg)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    st = scfft.OdeStats()
    scfft.scfft_integrate(s.ctx, 0.0, 0.03 * t0, h, scfft.default_ode_opts(), stats=st)
    torch.cuda.synchronize()
    from oracle import ode
    y, so = ode.integrate(lambda t, y: orhs.rhs_eval(prob, t, y), 0.0, 0.03 * t0 / u.t0,
                          np.zeros((3,) + prob.grid.shape), breakpoints=prob.drive.breakpoints())
    assert st.accepted > 5
    assert (st.accepted, st.rejected, st.rhs_calls) == (so.accepted, so.rejected, so.rhs_calls)
    assert rel_max(_np(h), y) < 1e-10


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("fuse", [2, 0])
@pytest.mark.parametrize("fixed", [3, 0])
def test_box_pruning_is_exact(prec, fuse, fixed):
    """Skipping the work outside Omega's bounding box changes nothing: the
    skipped inputs are exact zeros and the skipped outputs are never read."""
    cfg = CUP64
    dtype = torch.float64 if prec == scfft.F64 else torch.float32
    h = to_dev(torch, state(cfg, seed=9), dtype)
    outs = []
    for prune in (1, 0):
        s = sim(cfg, precision=prec, fixed_iter=fixed, fuse_xy=fuse, prune_box=prune)
        res = []
        for t_s in (0.002, 0.0021):                     # second call: warm start
            o, _ = s.rhs_eval(t_s, h)
            res.append(o.clone())
        torch.cuda.synchronize()
        outs.append(res)
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("cfg", [CUBE32, NONCUBIC, small_cfg((48, 24, 32), (2.0, 1.0, 1.4), workloads.shape_cube(0.6))],
                         ids=["32", "16x32x64", "48x24x32"])
def test_stray_fraction(cfg, prec):
    """||(1-chi) j|| / ||chi j|| of j = C_s h against the oracle (FP64 1e-10,
    FP32 1e-5 relative), on a state and on the right-hand side's output."""
    s = sim(cfg, precision=prec, fixed_iter=3)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h = to_dev(torch, state(cfg, seed=7), dt)
    hn = _np(h)
    tol = 1e-10 if prec == scfft.F64 else 1e-5
    got = scfft.scfft_stray_fraction(s.ctx, h)
    want = readouts.stray_fraction(prob.grid, prob.chi, hn)
    assert abs(got - want) <= tol * want
    out, _ = s.rhs_eval(0.01, h)                     # a field with most current outside Omega
    got = scfft.scfft_stray_fraction(s.ctx, out)
    want = readouts.stray_fraction(prob.grid, prob.chi, _np(out))
    assert abs(got - want) <= tol * want


def _fp32_vs_fp64(cfg, t0_s, steps, dt_s, start):
    res = []
    for prec, dt in ((scfft.F64, torch.float64), (scfft.F32, torch.float32)):
        s = sim(cfg, precision=prec, fixed_iter=3)
        h = start(s, dt)
        ms = []
        scfft.scfft_integrate(s.ctx, t0_s, t0_s + steps * dt_s, h, scfft.default_ode_opts(fixed_steps=steps),
                              observer=lambda _u, t, _p: ms.append(scfft.scfft_step_moment(s.ctx)) or 0)
        j = s.empty_field()
        scfft.scfft_current(s.ctx, h, j)
        torch.cuda.synchronize()
        res.append((_np(h), _np(j), np.array(ms)))
    return res


def test_fp32_trajectory_against_fp64():
    """FP32 bulk path against FP64 along trajectories of the shield (64^3 box,
    n = 100, the 45-degree 50 Hz drive, 3 exterior iterations), within 1e-4
    relative L2:
      * from the virgin state, 60 fixed steps of 2e-5 s: h and j = C_s h at
        the end and the moment of every accepted state;
      * from a critical-state synthetic start at the peak field (|j| = 1.05
        in Omega, where the law is steepest), 20 steps: h and j at the end
        (the moment of that random current is a sum that cancels to 1e-3 of
        its terms, so FP32 rounding of j shows in it at that ratio)."""
    cfg = CUP64

    def virgin(s, dt):
        h = s.empty_field()
        scfft.scfft_init_state(s.ctx, 0.0, h)
        return h

    (h64, j64, m64), (h32, j32, m32) = _fp32_vs_fp64(cfg, 0.0, 60, 2e-5, virgin)
    assert m64.shape == (60, 3)
    assert rel_l2(h32, h64) < 1e-4 and rel_l2(j32, j64) < 1e-4 and rel_l2(m32, m64) < 1e-4
    print("virgin: FP32 vs FP64 rel L2 h %.2e j %.2e m %.2e" % (rel_l2(h32, h64), rel_l2(j32, j64),
                                                                 rel_l2(m32, m64)))

    def critical(s, dt):
        he, _ = scfft.scfft_drive_eval(s.drive, s.material, 0.005)
        return to_dev(torch, state(cfg, seed=0, bg=tuple(he)), dt)

    (h64, j64, _), (h32, j32, _) = _fp32_vs_fp64(cfg, 0.005, 20, 2e-5, critical)
    assert rel_l2(h32, h64) < 1e-4 and rel_l2(j32, j64) < 1e-4
    print("critical: FP32 vs FP64 rel L2 h %.2e j %.2e (rel max h %.2e j %.2e)"
          % (rel_l2(h32, h64), rel_l2(j32, j64), rel_max(h32, h64), rel_max(j32, j64)))


@pytest.mark.parametrize("cfg", [NONCUBIC, CUBE32], ids=["16x32x64", "32"])
def test_rhs_adaptive_iteration_guess(cfg):
    """The adaptive loop launches as many iterations as the previous call
    needed: calls needing more (a start from Ohm's law after a warm call),
    as many, and fewer than guessed all give the oracle's iteration count,
    last delta and result."""
    s = sim(cfg, delta_it=2e-5)
    prob, u = oracle_problem(cfg, delta_it=2e-5)
    h = state(cfg, seed=4)
    dh = to_dev(torch, h, torch.float64)
    seen = []
    for t_s, reset in ((0.2, False), (0.21, False), (0.215, False), (0.22, True), (0.23, False)):
        if reset:
            scfft.scfft_reset_warm(s.ctx)
            prob.warm = None
        stats = scfft.RhsStats()
        out, rc = s.rhs_eval(t_s, dh, stats=stats)
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        assert stats.iters == prob.last_iters, t_s
        assert abs(stats.last_delta - prob.last_deltas[-1]) <= 1e-9 * prob.last_deltas[-1]
        assert rel_max(_np(out), want) < 1e-10, t_s
        seen.append(stats.iters)
    assert seen[3] > seen[2]                              # the Ohm-law restart needed more than guessed


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_cube_axis_permutation_symmetry_on_gpu(prec):
    """A cube under a field along z and the same cube under the field along
    x with the state's x and z swapped (grid axes and components) give right-
    hand sides that map onto each other (P8): the X, Y and Z passes treat
    their axes alike."""
    base = small_cfg((32, 32, 32), (2.0, 2.0, 2.0), workloads.shape_cube(1.0), n_power=20.0)
    dt = torch.float64 if prec == scfft.F64 else torch.float32

    def swap(v):
        return np.ascontiguousarray(np.transpose(v[[2, 1, 0]], (0, 3, 2, 1)))

    def run(direction, h):
        cfg = dict(base, drive=dict(kind="ramp_hold", direction=direction, amp_T=0.1, t_ramp_s=1.0))
        s = sim(cfg, precision=prec, fixed_iter=4, fuse_xy=0)
        out, _ = s.rhs_eval(0.25, to_dev(torch, h, dt))
        torch.cuda.synchronize()
        return _np(out)

    hz = state(base, seed=6, bg=(0.0, 0.0, 0.1))
    a = run((0.0, 0.0, 1.0), hz)
    b = run((1.0, 0.0, 0.0), swap(hz))
    tol = 1e-11 if prec == scfft.F64 else 1e-5
    assert np.max(np.abs(swap(a) - b)) <= tol * np.max(np.abs(a))
