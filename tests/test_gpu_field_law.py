"""Field-dependent critical density (Kim-type e(j, h), allowed after Eq. 1)
on the GPU against the oracle: one right-hand side with both pass schedules,
a fixed-step integration (stage arguments formed inside the passes), FP32
against FP64, and the reverse mode refusing it."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, state, to_dev
from oracle import ode, rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUBE32 = dict(workloads.config("cube32"), n_power=20.0)
MU0 = 4e-7 * np.pi
B0, ALPHA = 0.2, 1.0


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


def _problem(cfg, **opt):
    prob, u = oracle_problem(cfg, **opt)
    prob.field_law = (B0 / (MU0 * cfg["jc"] * cfg["l_m"]), ALPHA)
    return prob, u


@pytest.mark.parametrize("fuse", [2, 0])
def test_rhs_field_law_fp64(fuse):
    cfg = CUBE32
    prob, u = _problem(cfg, fixed_iter=3)
    s = sim(cfg, fixed_iter=3, fuse_xy=fuse)
    scfft.scfft_set_field_law(s.ctx, B0, ALPHA)
    h = state(cfg, seed=4, bg=(0.0, 0.1, 0.3))
    out, _ = s.rhs_eval(0.01 * u.t0, to_dev(torch, h, torch.float64))
    want = orhs.rhs_eval(prob, 0.01, h)
    assert rel_max(out.cpu().numpy(), want) < 1e-10
    # the field law changes the result
    s0 = sim(cfg, fixed_iter=3, fuse_xy=fuse)
    plain, _ = s0.rhs_eval(0.01 * u.t0, to_dev(torch, h, torch.float64))
    assert rel_max(plain.cpu().numpy(), want) > 1e-3


def test_integrate_field_law_fp64():
    cfg = CUBE32
    prob, u = _problem(cfg, fixed_iter=2)
    s = sim(cfg, fixed_iter=2)
    scfft.scfft_set_field_law(s.ctx, B0, ALPHA)
    h0 = state(cfg, seed=5, bg=(0.0, 0.1, 0.3))
    h = to_dev(torch, h0, torch.float64)
    # the lowered critical density makes e large: a short horizon keeps the explicit steps stable
    scfft.scfft_integrate(s.ctx, 0.0, 2e-4, h, scfft.default_ode_opts(fixed_steps=4))
    torch.cuda.synchronize()
    y, _ = ode.integrate(lambda t, yy: orhs.rhs_eval(prob, t, yy), 0.0, 2e-4 / u.t0, h0, fixed_steps=4)
    assert np.all(np.isfinite(y)) and rel_max(y, h0) > 1e-6       # it moved
    assert rel_max(h.cpu().numpy(), y) < 1e-10


def test_field_law_fp32_and_reverse_mode():
    cfg = CUBE32
    h = state(cfg, seed=6, bg=(0.0, 0.1, 0.3))
    outs = []
    for prec, dt in ((scfft.F64, torch.float64), (scfft.F32, torch.float32)):
        s = sim(cfg, precision=prec, fixed_iter=3)
        scfft.scfft_set_field_law(s.ctx, B0, ALPHA)
        o, _ = s.rhs_eval(0.01, to_dev(torch, h, dt))
        torch.cuda.synchronize()
        outs.append(o.double().cpu().numpy())
        if prec == scfft.F64:
            hb = s.empty_field()
            dh = to_dev(torch, h, dt)
            with pytest.raises(scfft.ScfftError):
                scfft.scfft_rhs_vjp(s.ctx, dh, True, dh, None, hb)
            scfft.scfft_set_field_law(s.ctx, 0.0, 1.0)         # off again: accepted
            scfft.scfft_rhs_vjp(s.ctx, dh, True, dh, None, hb)
    assert rel_l2(outs[1], outs[0]) < 1e-4
