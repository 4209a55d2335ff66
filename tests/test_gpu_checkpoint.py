"""Checkpoint and resume: the state blob (warm start of iteration (5) and the
right-hand-side options) taken between two integration chunks lets a fresh
context continue exactly where the first one went on; blobs for another grid
or precision, or cut short, are refused."""
import numpy as np
import pytest

from gpu_case import rel_max, sim, small_cfg, state, to_dev
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUP = small_cfg((32, 32, 32), (2.0, 2.0, 2.0), workloads.shape_cup(1.0, 0.6, 2.0, 0.3), n_power=20.0)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("opt", [dict(fixed_iter=2), dict(delta_it=2e-5)], ids=["fixed", "adaptive"])
def test_resume_from_state_blob(opt):
    h0 = to_dev(torch, state(CUP, seed=3), torch.float64)
    o = scfft.default_ode_opts(fixed_steps=4)
    a = sim(CUP, **opt)
    h = h0.clone()
    scfft.scfft_integrate(a.ctx, 0.0, 0.01, h, o)
    blob = scfft.scfft_get_state(a.ctx)
    h_mid = h.clone()
    scfft.scfft_integrate(a.ctx, 0.01, 0.02, h, o)
    b = scfft.Simulation(CUP, precision=scfft.F64)           # default options until restored
    scfft.scfft_set_state(b.ctx, blob)
    hb = h_mid.clone()
    scfft.scfft_integrate(b.ctx, 0.01, 0.02, hb, o)
    torch.cuda.synchronize()
    if "fixed_iter" in opt:
        assert torch.equal(hb, h)                            # the same arithmetic
    else:
        assert rel_max(hb.cpu().numpy(), h.cpu().numpy()) < 1e-12
    # without the blob the continuation starts the exterior iteration afresh
    c = sim(CUP, **opt)
    hc = h_mid.clone()
    scfft.scfft_integrate(c.ctx, 0.01, 0.02, hc, o)
    torch.cuda.synchronize()
    assert not torch.equal(hc, h)


def test_state_blob_is_checked():
    a = sim(CUP, fixed_iter=2)
    h = to_dev(torch, state(CUP, seed=4), torch.float64)
    a.rhs_eval(0.01, h)
    blob = scfft.scfft_get_state(a.ctx)
    other = sim(small_cfg((32, 32, 16), (2.0, 2.0, 1.0), workloads.shape_cube(0.5)), fixed_iter=2)
    f32 = sim(CUP, precision=scfft.F32, fixed_iter=2)
    for ctx, b in ((other.ctx, blob), (f32.ctx, blob), (a.ctx, blob[:len(blob) // 2]),
                   (a.ctx, b"\0" * len(blob))):
        with pytest.raises(scfft.ScfftError) as e:
            scfft.scfft_set_state(ctx, b)
        assert e.value.status == scfft.ERR_STATE
    assert scfft.scfft_set_state(a.ctx, blob) == scfft.OK
