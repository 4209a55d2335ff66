"""Grids with axes of 3 * 2^k nodes (24, 48, 96, 192; one radix-3 pass in
each transform) against the oracle, which transforms such axes by the direct
DFT: the operators along each axis, the right-hand side in FP64 and FP32,
the reverse mode, and a few integrator steps.  Tolerances as for the
power-of-two grids: operators <= 1e-12, FP64 right-hand side <= 1e-10
(relative to the largest reference value), FP32 <= 1e-4 relative L2."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import adjoint, operators
from oracle import rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUP = workloads.shape_cup(1.0, 0.8, 2.0, 0.2)
C24 = small_cfg((24, 24, 24), (2.0, 2.0, 2.0), workloads.shape_cube(1.0))
C48 = small_cfg((48, 48, 48), (2.0, 2.0, 2.0), CUP)
MIXED = small_cfg((48, 32, 24), (2.0, 1.5, 1.2), workloads.shape_cylinder(0.8, 1.6, axis=0))
X192 = small_cfg((192, 24, 24), (4.0, 1.0, 1.0), workloads.shape_cylinder(0.5, 4.0, axis=0))
Y192 = small_cfg((24, 192, 24), (1.0, 4.0, 1.0), workloads.shape_cylinder(0.5, 4.0, axis=1))
Z192 = small_cfg((24, 24, 192), (1.0, 1.0, 4.0), workloads.shape_cylinder(0.5, 4.0, axis=2))
Y96 = small_cfg((16, 96, 48), (1.0, 3.0, 2.0), workloads.shape_cube(0.6))


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("cfg", [C24, MIXED, X192, Y192, Z192, Y96],
                         ids=["24", "48x32x24", "192x24x24", "24x192x24", "24x24x192", "16x96x48"])
def test_curl_and_phi(cfg, prec):
    s = sim(cfg, precision=prec)
    g, _ = oracle_problem(cfg)
    v = np.random.default_rng(1).normal(size=s.field_shape)     # full band, Nyquist included
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    dv = to_dev(torch, v, dt)
    vv = _np(dv)                                                # the input as the device holds it
    out = s.empty_field()
    for op, ref in ((scfft.scfft_curl, operators.curl_s), (scfft.scfft_phi, operators.phi)):
        op(s.ctx, dv, out)
        torch.cuda.synchronize()
        want = ref(vv, g.grid)
        if prec == scfft.F64:
            assert rel_max(_np(out), want) < 1e-12
        else:
            assert rel_l2(_np(out), want) < 1e-5


@pytest.mark.parametrize("cfg", [C24, C48, MIXED], ids=["24", "48", "48x32x24"])
def test_rhs_fixed_iter_fp64(cfg):
    s = sim(cfg, fixed_iter=3)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=2)
    dh = to_dev(torch, h, torch.float64)
    for t_s in (0.25, 0.3):                                    # the second uses the warm start
        out, _ = s.rhs_eval(t_s, dh)
        torch.cuda.synchronize()
        assert rel_max(_np(out), orhs.rhs_eval(prob, t_s / u.t0, h)) < 1e-10, t_s


def test_rhs_adaptive_fp64_and_fp32():
    cfg = C48
    prob, u = oracle_problem(cfg, delta_it=2e-5)
    h = state(cfg, seed=4)
    s = sim(cfg, delta_it=2e-5)
    st = scfft.RhsStats()
    out, _ = s.rhs_eval(0.2, to_dev(torch, h, torch.float64), stats=st)
    want = orhs.rhs_eval(prob, 0.2 / u.t0, h)
    assert st.iters == prob.last_iters
    assert rel_max(_np(out), want) < 1e-10
    s32 = sim(cfg, precision=scfft.F32, fixed_iter=3)
    prob3, _ = oracle_problem(cfg, fixed_iter=3)
    out32, _ = s32.rhs_eval(0.2, to_dev(torch, h, torch.float32))
    torch.cuda.synchronize()
    assert rel_l2(_np(out32), orhs.rhs_eval(prob3, 0.2 / u.t0, h)) < 1e-4


def test_rhs_vjp_fp64():
    cfg = MIXED
    prob, u = oracle_problem(cfg, fixed_iter=2)
    s = sim(cfg, fixed_iter=2)
    h = state(cfg, seed=6)
    j = operators.curl_s(h, prob.grid)
    a = np.sqrt(np.sum(j * j, axis=0))[prob.chi != 0]
    h = h * (1.05 / float(np.max(a)))                          # the law is active in Omega
    lam = state(cfg, seed=7, bg=(0.0, 0.0, 0.0))
    mu = state(cfg, seed=8, bg=(0.0, 0.0, 0.0))
    hbar, wbar = s.empty_field(), s.empty_field()
    nb, hb = scfft.scfft_rhs_vjp(s.ctx, to_dev(torch, h, torch.float64), True, to_dev(torch, lam, torch.float64),
                                 to_dev(torch, mu, torch.float64), hbar, wbar)
    torch.cuda.synchronize()
    r = adjoint.rhs_vjp(prob, 0.01, h, True, lam, mu)
    assert rel_max(_np(hbar), r["h_bar"]) < 1e-10
    assert rel_max(_np(wbar), r["w_bar"]) < 1e-10
    assert abs(nb - r["n_bar"]) <= 1e-10 * abs(r["n_bar"])


def test_integrate_fixed_steps_fp64_and_graph():
    cfg = C48
    prob, u = oracle_problem(cfg, fixed_iter=2)
    h0 = state(cfg, seed=9)
    steps, t1_s = 3, 0.01
    s = sim(cfg, fixed_iter=2)
    h = to_dev(torch, h0, torch.float64)
    scfft.scfft_integrate(s.ctx, 0.0, t1_s, h, scfft.default_ode_opts(fixed_steps=steps))
    torch.cuda.synchronize()
    # the oracle's fixed-step BS23 over the same steps
    from oracle import ode
    y, _ = ode.integrate(lambda t, y: orhs.rhs_eval(prob, t, y), 0.0, t1_s / u.t0, h0, fixed_steps=steps)
    assert rel_max(_np(h), y) < 1e-10
    g = sim(cfg, fixed_iter=2)
    hg = to_dev(torch, h0, torch.float64)
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(g.ctx, steps))
    scfft.scfft_integrate_graph(g.ctx, 0.0, t1_s, steps, ws, hg)
    scfft.scfft_integrate_wait(g.ctx, scfft.OdeStats())
    torch.cuda.synchronize()
    assert rel_max(_np(hg), _np(h)) < 1e-12
