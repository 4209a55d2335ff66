"""The fixed-step integrator, which enqueues the next step before it waits
for the current one's error norm: the state after an observer stops the run
is the state of that many steps, a non-finite state stops it with the last
accepted state in h, and the observer's step moments equal the stand-alone
readout of each state it is shown."""
import numpy as np
import pytest

from gpu_case import sim, state, to_dev
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUBE32 = dict(workloads.config("cube32"), n_power=20.0)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_observer_stop_gives_the_state_of_that_many_steps(prec):
    cfg = CUBE32
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h0 = to_dev(torch, state(cfg, seed=31), dt)
    t1, steps, stop_at = 0.006, 6, 3
    a = sim(cfg, precision=prec, fixed_iter=2)
    ha = h0.clone()
    seen = []

    def obs(_u, t, p):
        seen.append(t)
        return 1 if len(seen) == stop_at else 0

    st = scfft.OdeStats()
    scfft.scfft_integrate(a.ctx, 0.0, t1, ha, scfft.default_ode_opts(fixed_steps=steps), observer=obs, stats=st)
    assert len(seen) == stop_at and st.accepted == stop_at
    assert abs(st.t_s - stop_at * t1 / steps) <= 1e-12 * t1
    # the same step size, stop_at steps, on a fresh context (same start, no warm start)
    b = sim(cfg, precision=prec, fixed_iter=2)
    hb = h0.clone()
    scfft.scfft_integrate(b.ctx, 0.0, stop_at * t1 / steps, hb, scfft.default_ode_opts(fixed_steps=stop_at))
    torch.cuda.synchronize()
    # step sizes agree to rounding ((t1 / 6) against (t1 / 2) / 3)
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    ref = hb.double()
    assert float((ha.double() - ref).abs().max()) <= tol * float(ref.abs().max())
    assert float((ha.double() - h0.double()).abs().max()) > 1e-6 * float(ref.abs().max())   # it moved


def test_non_finite_state_keeps_the_last_accepted_state():
    cfg = CUBE32
    s = sim(cfg, fixed_iter=2)
    h0 = to_dev(torch, state(cfg, seed=32), torch.float64)
    # a field that a few steps drive to overflow: huge and with a steep law
    big = h0 * 1e150
    h = big.clone()
    st = scfft.OdeStats()
    with pytest.raises(scfft.ScfftError) as ei:
        scfft.scfft_integrate(s.ctx, 0.0, 0.01, h, scfft.default_ode_opts(fixed_steps=4), stats=st)
    assert ei.value.status == scfft.ERR_NAN
    torch.cuda.synchronize()
    assert bool(torch.isfinite(h).all())                  # the last accepted state
    if st.accepted == 0:
        assert torch.equal(h, big)


@pytest.mark.parametrize("fuse", [0, 2])
def test_step_moments_match_the_readout_of_each_observed_state(fuse):
    cfg = CUBE32
    s = sim(cfg, fixed_iter=2, fuse_xy=fuse)
    h = to_dev(torch, state(cfg, seed=33), torch.float64)
    got = []

    def obs(_u, t, p):
        got.append((scfft.scfft_step_moment(s.ctx, 0), scfft.scfft_moment(s.ctx, p, 0),
                    scfft.scfft_step_moment(s.ctx, 1), scfft.scfft_moment(s.ctx, p, 1)))
        return 0

    scfft.scfft_integrate(s.ctx, 0.0, 0.005, h, scfft.default_ode_opts(fixed_steps=5), observer=obs)
    assert len(got) == 5
    for m_all, r_all, m_in, r_in in got:
        assert np.max(np.abs(m_all - r_all)) <= 1e-12 * np.max(np.abs(r_all))
        assert np.max(np.abs(m_in - r_in)) <= 1e-12 * np.max(np.abs(r_in))
