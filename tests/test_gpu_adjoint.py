"""Reverse mode on the GPU against the oracle's reverse mode (itself pinned by
the affine-case adjoint identity and central differences): one
right-hand-side call (fixed iteration count, explicit warm start) and the
fixed-step integrator with checkpoints.  FP64 <= 1e-10 relative to the
largest reference value; FP32 against FP64 <= 1e-4 relative L2."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import adjoint, operators
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUBE32 = dict(workloads.config("cube32"), n_power=20.0)
NONCUBIC = small_cfg((16, 32, 64), (1.5, 2.0, 3.0), workloads.shape_cup(1.0, 0.6, 3.0, 0.4, axis=1))
SQZ = small_cfg((32, 32, 16), (2.0, 2.0, 1.0), workloads.shape_cylinder(0.8, 1.2))


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


def _scaled_state(cfg, prob, seed, bg=(0.0, 0.02, 0.05)):
    """State whose smoothed current reaches 1.05 in Omega."""
    h = state(cfg, seed=seed, bg=(0.0, 0.0, 0.0))
    j = operators.curl_s(h, prob.grid)
    a = np.sqrt(np.sum(j * j, axis=0))[prob.chi != 0]
    return h * (1.05 / float(np.max(a))) + np.asarray(bg).reshape(3, 1, 1, 1)


def _kappa(cfg, seed):
    n = cfg["n"]
    return 1.0 + 0.1 * np.random.default_rng(seed).normal(size=(n[2], n[1], n[0]))


def _rel(x, r):
    return abs(x - r) / max(abs(r), 1e-300)


@pytest.mark.parametrize("cfg", [CUBE32, NONCUBIC], ids=["cube32", "noncubic"])
@pytest.mark.parametrize("warm_used", [True, False])
@pytest.mark.parametrize("with_kappa", [False, True])
def test_rhs_vjp_fp64(cfg, warm_used, with_kappa):
    K = 3
    prob, u = oracle_problem(cfg, fixed_iter=K)
    s = sim(cfg, fixed_iter=K)
    kap = _kappa(cfg, 4) if with_kappa else None
    if kap is not None:
        prob.kappa = kap
        dk = to_dev(torch, kap, torch.float64)
        scfft.scfft_set_jc_map(s.ctx, dk)
    h = _scaled_state(cfg, prob, 1)
    lam = state(cfg, seed=2, bg=(0.0, 0.0, 0.0))
    mu = state(cfg, seed=3, bg=(0.0, 0.0, 0.0))
    dh, dl, dm = (to_dev(torch, a, torch.float64) for a in (h, lam, mu))
    hbar, wbar = s.empty_field(), s.empty_field()
    kbar = torch.zeros(prob.grid.shape, dtype=torch.float64, device="cuda")
    nb, hb = scfft.scfft_rhs_vjp(s.ctx, dh, warm_used, dl, dm, hbar, wbar, kbar)
    torch.cuda.synchronize()
    r = adjoint.rhs_vjp(prob, 0.01, h, warm_used, lam, mu)
    assert rel_max(_np(hbar), r["h_bar"]) < 1e-10
    assert rel_max(_np(wbar), r["w_bar"]) < 1e-10
    assert rel_max(_np(kbar), r["kappa_bar"]) < 1e-10
    assert _rel(nb, r["n_bar"]) < 1e-10
    assert np.max(np.abs(hb - r["hedot_bar"])) <= 1e-10 * np.max(np.abs(r["hedot_bar"]))


def test_rhs_with_kappa_map_fp64():
    """Forward right-hand side with a local critical-density map (Eq. 1 with
    jc(x)) against the oracle."""
    cfg = CUBE32
    prob, u = oracle_problem(cfg, fixed_iter=3)
    s = sim(cfg, fixed_iter=3)
    prob.kappa = _kappa(cfg, 5)
    scfft.scfft_set_jc_map(s.ctx, to_dev(torch, prob.kappa, torch.float64))
    h = _scaled_state(cfg, prob, 6)
    out, _ = s.rhs_eval(0.01 * u.t0, to_dev(torch, h, torch.float64))
    want = adjoint.rhs_forward(prob, 0.01, h, None)[0]
    assert rel_max(_np(out), want) < 1e-10


def test_rhs_vjp_fp32_vs_fp64():
    cfg = CUBE32
    prob, _ = oracle_problem(cfg, fixed_iter=3)
    h = _scaled_state(cfg, prob, 7)
    lam = state(cfg, seed=8, bg=(0.0, 0.0, 0.0))
    mu = state(cfg, seed=9, bg=(0.0, 0.0, 0.0))
    res = []
    for prec, dt in ((scfft.F64, torch.float64), (scfft.F32, torch.float32)):
        s = sim(cfg, precision=prec, fixed_iter=3)
        hbar, wbar = s.empty_field(), s.empty_field()
        nb, hb = scfft.scfft_rhs_vjp(s.ctx, to_dev(torch, h, dt), True, to_dev(torch, lam, dt),
                                     to_dev(torch, mu, dt), hbar, wbar)
        torch.cuda.synchronize()
        res.append((_np(hbar), _np(wbar), nb, hb))
    (a, b, n64, h64), (c, d, n32, h32) = res
    assert rel_l2(c, a) < 1e-4 and rel_l2(d, b) < 1e-4
    assert _rel(n32, n64) < 1e-4
    assert np.max(np.abs(h32 - h64)) <= 1e-4 * np.max(np.abs(h64))


def _adjoint_run(s, cfg, h0, hT_bar, steps, every, t1_s, dtype=torch.float64, kbar=None):
    nbytes = scfft.scfft_adjoint_workspace_size(s.ctx, steps, every)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + nbytes]
    hT, h0b = s.empty_field(), s.empty_field()
    nb, pb = scfft.scfft_integrate_adjoint(s.ctx, 0.0, t1_s, steps, every, ws, to_dev(torch, h0, dtype),
                                           to_dev(torch, hT_bar, dtype), hT, h0b, kbar)
    torch.cuda.synchronize()
    return hT, h0b, nb, pb


@pytest.mark.parametrize("cfg", [SQZ, NONCUBIC], ids=["sqz", "noncubic"])
def test_integrate_adjoint_fp64(cfg):
    K, steps, every = 2, 5, 2          # three segments, the last one ragged
    prob, u = oracle_problem(cfg, fixed_iter=K)
    s = sim(cfg, fixed_iter=K)
    h0 = _scaled_state(cfg, prob, 11)
    ybar = state(cfg, seed=12, bg=(0.0, 0.0, 0.0))
    t1_s = 2e-3 * u.t0
    kbar = torch.zeros(prob.grid.shape, dtype=torch.float64, device="cuda")
    hT, h0b, nb, pb = _adjoint_run(s, cfg, h0, ybar, steps, every, t1_s, kbar=kbar)
    yT, g = adjoint.integrate_adjoint(prob, 0.0, t1_s / u.t0, h0, steps, ybar)
    assert rel_max(_np(hT), yT) < 1e-10
    assert rel_max(_np(h0b), g["y0_bar"]) < 1e-10
    assert rel_max(_np(kbar), g["kappa_bar"]) < 1e-10
    assert _rel(nb, g["n_bar"]) < 1e-10
    assert np.max(np.abs(pb - g["p_bar"])) <= 1e-10 * np.max(np.abs(g["p_bar"]))


@pytest.mark.parametrize("fuse", [0, 2])
def test_integrate_adjoint_checkpoint_interval_and_forward_agree(fuse):
    """Any checkpoint interval gives bitwise the same gradient (the recomputed
    segments repeat the forward arithmetic, and where the tape holds no j the
    reverse call recomputes it with the forward call's pass schedule), and the
    forward result is that of scfft_integrate's fixed-step mode after a
    warm-start reset."""
    cfg = SQZ
    prob, u = oracle_problem(cfg, fixed_iter=2)
    s = sim(cfg, fixed_iter=2, fuse_xy=fuse)
    h0 = _scaled_state(cfg, prob, 13)
    ybar = state(cfg, seed=14, bg=(0.0, 0.0, 0.0))
    t1_s, steps = 2e-3 * u.t0, 6
    outs = [_adjoint_run(s, cfg, h0, ybar, steps, every, t1_s) for every in (1, 4, 6, 50)]
    for hT, h0b, nb, pb in outs[1:]:
        assert torch.equal(hT, outs[0][0]) and torch.equal(h0b, outs[0][1])
        assert nb == outs[0][2] and np.array_equal(pb, outs[0][3])
    scfft.scfft_reset_warm(s.ctx)
    h = to_dev(torch, h0, torch.float64)
    scfft.scfft_integrate(s.ctx, 0.0, t1_s, h, scfft.default_ode_opts(fixed_steps=steps))
    torch.cuda.synchronize()
    assert torch.equal(h, outs[0][0])


def test_integrate_adjoint_fp32_vs_fp64():
    cfg = SQZ
    prob, u = oracle_problem(cfg, fixed_iter=2)
    h0 = _scaled_state(cfg, prob, 15)
    ybar = state(cfg, seed=16, bg=(0.0, 0.0, 0.0))
    res = []
    for prec, dt in ((scfft.F64, torch.float64), (scfft.F32, torch.float32)):
        s = sim(cfg, precision=prec, fixed_iter=2)
        hT, h0b, nb, pb = _adjoint_run(s, cfg, h0, ybar, 4, 2, 2e-3 * u.t0, dtype=dt)
        res.append((_np(hT), _np(h0b), nb, pb))
    assert rel_l2(res[1][0], res[0][0]) < 1e-4
    assert rel_l2(res[1][1], res[0][1]) < 1e-4
    assert _rel(res[1][2], res[0][2]) < 1e-4


def test_reverse_mode_argument_errors():
    cfg = SQZ
    s = sim(cfg)                                    # adaptive iteration: no reverse mode
    h = s.empty_field().zero_()
    hb = s.empty_field()
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_rhs_vjp(s.ctx, h, True, h, None, hb)
    s2 = sim(cfg, fixed_iter=2)
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_rhs_vjp(s2.ctx, h, True, h, None, h)           # output aliases input
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_integrate_adjoint(s2.ctx, 0.0, 1.0, 4, 2, small, h, h, None, hb)


def test_autograd_gradcheck():
    """torch.autograd.gradcheck (central differences of the GPU forward path
    against the library's reverse mode) for one call and for the integrator."""
    from paper_1803_01346_amd import autograd as sag
    cfg = small_cfg((8, 8, 8), (1.0, 1.0, 1.0), workloads.shape_cube(0.5))
    prob, u = oracle_problem(cfg, fixed_iter=2)
    s = sim(cfg, fixed_iter=2)
    h = to_dev(torch, _scaled_state(cfg, prob, 21), torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: sag.RhsEval.apply(x, s, 0.01 * u.t0), (h,), eps=1e-6,
                                    atol=1e-6, rtol=1e-4, fast_mode=True)
    assert torch.autograd.gradcheck(lambda x: sag.Integrate.apply(x, s, 0.0, 1e-3 * u.t0, 3, 2), (h,),
                                    eps=1e-6, atol=1e-6, rtol=1e-4, fast_mode=True)


def test_parameter_gradients_against_central_differences():
    """The shield-type loss L = mean over the bore of |h(t1)|^2 after fixed
    steps of a 45-degree field ramp that drives the cup wall to the critical
    state (|j| near 1, so n and kappa matter), differentiated by one adjoint run
    (IntegrateParams) with respect to a global jc (uniform scaling of the
    kappa map), one kappa voxel, n and the field angle, against central
    differences of the GPU forward path with relative step 1e-6: within
    1e-4 relative."""
    import math
    from paper_1803_01346_amd import autograd as sag
    theta = math.pi / 4
    l, jc = 5e-3, 1e8
    t0 = 4e-7 * math.pi * jc * l * l / 1e-4
    h_end = 0.3                                           # ramp rate h_e' = 1 up to 0.3
    base = small_cfg((32, 32, 32), (2.0, 2.0, 2.0), workloads.shape_cup(1.0, 0.6, 2.0, 0.3), n_power=20.0,
                     l_m=l, jc=jc,
                     drive=dict(kind="ramp_hold", direction=(math.sin(theta), 0.0, math.cos(theta)),
                                amp_T=h_end * 4e-7 * math.pi * jc * l, t_ramp_s=h_end * t0))
    steps, every, t1_s = 150, 30, h_end * t0              # dt' = 2e-3: stable for the explicit pair
    prob, _ = oracle_problem(base)
    g = prob.grid
    x = -2.0 + (np.arange(32) + 0.5) * (4.0 / 32)
    r = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2) * np.ones((32, 32, 32))
    bore = torch.from_numpy(((r < 0.5) & (np.abs(x)[:, None, None] < 0.6) & (prob.chi == 0))
                            .astype(np.float64)).cuda()
    nb = float(bore.sum())
    kap0 = torch.from_numpy(_kappa(base, 9)).cuda()
    h0 = torch.zeros((3, 32, 32, 32), dtype=torch.float64, device="cuda")

    def make(n_power):
        return sim(dict(base, n_power=n_power), fixed_iter=2)

    s = make(20.0)
    p0 = sag.drive_vector(s)
    amp = float(torch.linalg.norm(p0))

    def loss(sim_, kap, p):
        nt_ = torch.tensor(float(sim_.cfg["n_power"]), dtype=torch.float64)
        hT = sag.IntegrateParams.apply(h0, kap, nt_, p, sim_, 0.0, t1_s, steps, every)
        return (hT * hT).sum(dim=0).mul(bore).sum() / nb

    kap = kap0.clone().requires_grad_(True)
    nt = torch.tensor(20.0, dtype=torch.float64, requires_grad=True)
    pt = p0.clone().requires_grad_(True)
    L = sag.IntegrateParams.apply(h0, kap, nt, pt, s, 0.0, t1_s, steps, every)
    L = (L * L).sum(dim=0).mul(bore).sum() / nb
    L.backward()
    kbar, n_bar, p_bar = kap.grad, float(nt.grad), pt.grad.double().cpu().numpy()
    eps = 1e-6

    def rel(a, b):
        return abs(a - b) / max(abs(b), 1e-300)

    with torch.no_grad():
        # global jc: kappa -> (1 + e) kappa
        fd = (float(loss(s, kap0 * (1 + eps), p0)) - float(loss(s, kap0 * (1 - eps), p0))) / (2 * eps)
        assert rel(float((kbar * kap0).sum()), fd) < 1e-4
        # the voxel of the map with the largest sensitivity
        iz, iy, ix = np.unravel_index(int(torch.argmax(kbar.abs())), kbar.shape)
        dk = torch.zeros_like(kap0)
        dk[iz, iy, ix] = eps * float(kap0[iz, iy, ix])
        fd = (float(loss(s, kap0 + dk, p0)) - float(loss(s, kap0 - dk, p0))) / (2 * float(dk[iz, iy, ix]))
        assert rel(float(kbar[iz, iy, ix]), fd) < 1e-4
        # n (a context per value of n)
        fd = (float(loss(make(20.0 * (1 + eps)), kap0, p0)) -
              float(loss(make(20.0 * (1 - eps)), kap0, p0))) / (2 * 20.0 * eps)
        assert rel(n_bar, fd) < 1e-4
        # field angle in the x-z plane
        def p_of(th):
            return torch.tensor([amp * math.sin(th), 0.0, amp * math.cos(th)], dtype=torch.float64)
        fd = (float(loss(s, kap0, p_of(theta + eps))) - float(loss(s, kap0, p_of(theta - eps)))) / (2 * eps)
        dth = float(np.dot(p_bar, [amp * math.cos(theta), 0.0, -amp * math.sin(theta)]))
        assert rel(dth, fd) < 1e-4


def test_config5_gradients_against_central_differences():
    """The adjoint configuration at full size: the 128^3 shield with a jc map
    kappa = 1 + 0.1 N(0,1) (seed 5), a critical-state start, 2000 fixed
    steps of 2e-5 s (checkpoints every 50), loss = mean over the bore of
    |h(t_end)|^2.  The gradients in n, in a global jc (a uniform scaling of
    kappa), in the field angle (the applied field turned in the x-z plane)
    and in the kappa voxel of largest sensitivity, all from one adjoint run,
    agree with central differences of the forward path (relative step 1e-6)
    within 1e-4."""
    import math
    from paper_1803_01346_amd import autograd as sag
    cfg = workloads.config("cup128")
    steps, every, t1_s = 2000, 50, 2000 * 2e-5
    n = cfg["n"]
    kap0 = torch.from_numpy(1.0 + 0.1 * np.random.default_rng(5).normal(size=(n[2], n[1], n[0]))).cuda()
    x = -4.0 + (np.arange(n[0]) + 0.5) * (8.0 / n[0])
    r = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2) * np.ones((n[2], n[1], n[0]))
    bore = torch.from_numpy(((r < 0.7) & (np.abs(x)[:, None, None] < 1.5)).astype(np.float64)).cuda()
    nb = float(bore.sum())

    def make(n_power):
        return sim(dict(cfg, n_power=n_power), fixed_iter=3)

    s = make(cfg["n_power"])
    he, _ = scfft.scfft_drive_eval(s.drive, s.material, 0.005)
    h0 = to_dev(torch, state(cfg, seed=0, bg=tuple(he)), torch.float64)
    p0 = sag.drive_vector(s)
    amp = float(torch.linalg.norm(p0))
    d = cfg["drive"]["direction"]
    theta = math.atan2(d[0], d[2])                         # angle from the z axis in the x-z plane
    assert abs(d[1]) < 1e-15

    def p_of(th):
        return torch.tensor([amp * math.sin(th), 0.0, amp * math.cos(th)], dtype=torch.float64)

    def loss(sim_, kap, p=p0):
        nt = torch.tensor(float(sim_.cfg["n_power"]), dtype=torch.float64)
        hT = sag.IntegrateParams.apply(h0, kap, nt, p, sim_, 0.0, t1_s, steps, every)
        return (hT * hT).sum(dim=0).mul(bore).sum() / nb

    kap = kap0.clone().requires_grad_(True)
    nt = torch.tensor(float(cfg["n_power"]), dtype=torch.float64, requires_grad=True)
    pt = p0.clone().requires_grad_(True)
    hT = sag.IntegrateParams.apply(h0, kap, nt, pt, s, 0.0, t1_s, steps, every)
    L = (hT * hT).sum(dim=0).mul(bore).sum() / nb
    L.backward()
    kbar = kap.grad
    g_jc, g_n = float((kbar * kap0).sum()), float(nt.grad)
    g_th = float(torch.dot(pt.grad.double().cpu(), torch.tensor(
        [amp * math.cos(theta), 0.0, -amp * math.sin(theta)], dtype=torch.float64)))
    iz, iy, ix = np.unravel_index(int(torch.argmax(kbar.abs())), kbar.shape)
    g_vox = float(kbar[iz, iy, ix])
    eps = 1e-6
    with torch.no_grad():
        fd_jc = (float(loss(s, kap0 * (1 + eps))) - float(loss(s, kap0 * (1 - eps)))) / (2 * eps)
        n0 = cfg["n_power"]
        fd_n = (float(loss(make(n0 * (1 + eps)), kap0)) - float(loss(make(n0 * (1 - eps)), kap0))) / (2 * n0 * eps)
        fd_th = (float(loss(s, kap0, p_of(theta + eps))) - float(loss(s, kap0, p_of(theta - eps)))) / (2 * eps)
        dk = torch.zeros_like(kap0)
        dk[iz, iy, ix] = eps * float(kap0[iz, iy, ix])
        fd_vox = (float(loss(s, kap0 + dk)) - float(loss(s, kap0 - dk))) / (2 * float(dk[iz, iy, ix]))
    print("dL/dln(jc) adjoint %.9e fd %.9e; dL/dn adjoint %.9e fd %.9e" % (g_jc, fd_jc, g_n, fd_n))
    print("dL/dtheta adjoint %.9e fd %.9e; dL/dkappa[%d,%d,%d] adjoint %.9e fd %.9e"
          % (g_th, fd_th, iz, iy, ix, g_vox, fd_vox))
    assert abs(g_jc - fd_jc) <= 1e-4 * abs(fd_jc)
    assert abs(g_n - fd_n) <= 1e-4 * abs(fd_n)
    assert abs(g_th - fd_th) <= 1e-4 * abs(fd_th)
    assert abs(g_vox - fd_vox) <= 1e-4 * abs(fd_vox)
    assert math.isfinite(float(L.detach()))
