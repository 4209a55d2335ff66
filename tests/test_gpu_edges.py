"""Edge cases against the oracle: the longest transforms (512 nodes along each
axis, one axis at a time), and the degenerate masks of the method: an empty
Omega (the exterior iteration returns the applied rate everywhere), Omega
filling the whole box (no exterior: the right-hand side is -C_s e), and a
single node."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import operators
from oracle import rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("n", [(512, 8, 8), (8, 512, 8), (8, 8, 512)], ids=["x512", "y512", "z512"])
def test_longest_transforms(n, prec):
    L = tuple(0.25 * v / 8 for v in n)                   # equal cells
    cfg = small_cfg(n, L, workloads.shape_cube(0.1))
    s = sim(cfg, precision=prec)
    prob, _ = oracle_problem(cfg)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    dv = to_dev(torch, np.random.default_rng(3).normal(size=s.field_shape), dt)
    vv = _np(dv)
    out = s.empty_field()
    for op, ref in ((scfft.scfft_curl, operators.curl_s), (scfft.scfft_phi, operators.phi)):
        op(s.ctx, dv, out)
        torch.cuda.synchronize()
        want = ref(vv, prob.grid)
        if prec == scfft.F64:
            assert rel_max(_np(out), want) < 1e-12
        else:
            assert rel_l2(_np(out), want) < 1e-5


def _with_mask(cfg, mask, **opt):
    s = sim(cfg, **opt)
    st = scfft.scfft_set_mask(s.ctx, torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).cuda())
    prob, u = oracle_problem(cfg, **opt)
    prob.chi = np.ascontiguousarray(mask, dtype=np.uint8)
    return s, prob, u, st


@pytest.mark.parametrize("opt", [dict(delta_it=2e-5), dict(fixed_iter=2)], ids=["adaptive", "fixed"])
def test_degenerate_masks(opt):
    cfg = small_cfg((16, 16, 16), (1.0, 1.0, 1.0), workloads.shape_cube(0.5),
                    drive=dict(kind="ramp_hold", direction=(0.3, -0.2, 1.0), amp_T=0.1, t_ramp_s=1.0))
    h = state(cfg, seed=8)
    shape = (16, 16, 16)
    one = np.zeros(shape, np.uint8)
    one[7, 8, 9] = 1
    for name, mask in (("empty", np.zeros(shape, np.uint8)), ("full", np.ones(shape, np.uint8)),
                       ("one node", one)):
        s, prob, u, st = _with_mask(cfg, mask, **opt)
        assert st == scfft.OK, name
        out, _ = s.rhs_eval(0.25, to_dev(torch, h, torch.float64))
        torch.cuda.synchronize()
        want = orhs.rhs_eval(prob, 0.25 / u.t0, h)
        assert rel_max(_np(out), want) < 1e-10, name
        if name == "empty":                              # the applied rate everywhere
            hedot = np.asarray(prob.drive.hedot(0.25 / u.t0)).reshape(3, 1, 1, 1)
            assert np.max(np.abs(_np(out) - hedot)) <= 1e-12 * np.max(np.abs(hedot))
        if name == "full":                               # no exterior: -C_s e
            e = _np(out)
            assert np.isfinite(e).all()
