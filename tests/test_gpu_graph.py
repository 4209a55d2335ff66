"""Graph-replayed fixed-step integration: the same trajectory as the plain
fixed-step integrator (which is pinned to the oracle), the non-finite stop,
the busy-context rule, and independent contexts on separate streams (the
batched use) giving what each gives alone."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_max, sim, small_cfg, state, to_dev
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CUBE32 = dict(workloads.config("cube32"), n_power=20.0)
SQZ = small_cfg((32, 32, 16), (2.0, 2.0, 1.0), workloads.shape_cylinder(0.8, 1.2))
NONCUBIC = small_cfg((16, 32, 64), (1.5, 2.0, 3.0), workloads.shape_cup(1.0, 0.6, 3.0, 0.4, axis=1))


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


def _graph_run(s, h, t1_s, steps):
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(s.ctx, steps))
    st = scfft.OdeStats()
    scfft.scfft_integrate_graph(s.ctx, 0.0, t1_s, steps, ws, h)
    scfft.scfft_integrate_wait(s.ctx, st)
    return st


@pytest.mark.parametrize("prec,fuse", [(scfft.F64, 0), (scfft.F64, 2), (scfft.F32, 1)])
def test_graph_matches_plain_fixed_steps(prec, fuse):
    cfg = CUBE32
    _, u = oracle_problem(cfg)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h0 = to_dev(torch, state(cfg, seed=1, bg=(0.0, 0.01, 0.02)), dt)
    t1_s, steps = 0.02, 7
    a = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=fuse)
    ha = h0.clone()
    sa = scfft.OdeStats()
    scfft.scfft_integrate(a.ctx, 0.0, t1_s, ha, scfft.default_ode_opts(fixed_steps=steps), stats=sa)
    b = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=fuse)
    hb = h0.clone()
    sb = _graph_run(b, hb, t1_s, steps)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    assert rel_max(hb.double().cpu().numpy(), ha.double().cpu().numpy()) < tol
    assert sb.accepted == steps and sb.rhs_calls == sa.rhs_calls
    assert abs(sb.t_s - sa.t_s) <= 1e-12 * sa.t_s
    assert abs(sb.err_last - sa.err_last) <= 1e-6 * abs(sa.err_last)
    # the context is usable again, and a second graph run continues the same way
    scfft.scfft_rhs_eval(b.ctx, 0.0, hb, b.empty_field())


def test_graph_stops_at_non_finite_error():
    cfg = SQZ
    s = sim(cfg, fixed_iter=2)
    h0 = to_dev(torch, state(cfg, seed=2), torch.float64)
    h0[1, 3, 5, 7] = float("nan")
    h = h0.clone()
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(s.ctx, 5))
    scfft.scfft_integrate_graph(s.ctx, 0.0, 0.01, 5, ws, h)
    with pytest.raises(scfft.ScfftError):              # busy until the wait
        scfft.scfft_rhs_eval(s.ctx, 0.0, h0, s.empty_field())
    st = scfft.OdeStats()
    with pytest.raises(scfft.ScfftError) as ei:
        scfft.scfft_integrate_wait(s.ctx, st)
    assert ei.value.status == scfft.ERR_NAN
    assert st.accepted == 0
    same = (h == h0) | (torch.isnan(h) & torch.isnan(h0))
    assert bool(same.all())                               # the last accepted state: the start
    with pytest.raises(scfft.ScfftError):                 # nothing left to wait for
        scfft.scfft_integrate_wait(s.ctx, st)


def test_graph_needs_fixed_iterations_and_workspace():
    cfg = SQZ
    s = sim(cfg)                                          # adaptive iteration
    h = s.empty_field().zero_()
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(s.ctx, 3))
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_integrate_graph(s.ctx, 0.0, 0.01, 3, ws, h)
    s2 = sim(cfg, fixed_iter=2)
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_integrate_graph(s2.ctx, 0.0, 0.01, 3, ws[:64], h)


def test_batched_contexts_on_streams():
    """Three instances of different sizes enqueued on their own streams, then
    waited for: each equals its own run alone (bitwise)."""
    cfgs = [CUBE32, SQZ, NONCUBIC]
    steps, t1_s = 4, 0.01
    alone = []
    for i, cfg in enumerate(cfgs):
        s = sim(cfg, fixed_iter=2)
        h = to_dev(torch, state(cfg, seed=10 + i), torch.float64)
        _graph_run(s, h, t1_s, steps)
        torch.cuda.synchronize()
        alone.append(h)
    streams = [torch.cuda.Stream() for _ in cfgs]
    sims, hs, wss = [], [], []
    for i, cfg in enumerate(cfgs):
        s = scfft.Simulation(cfg, precision=scfft.F64, stream=streams[i].cuda_stream,
                             rhs_opts=scfft.default_rhs_opts(fixed_iter=2))
        h = to_dev(torch, state(cfg, seed=10 + i), torch.float64)
        torch.cuda.synchronize()
        ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(s.ctx, steps))
        torch.cuda.synchronize()
        scfft.scfft_integrate_graph(s.ctx, 0.0, t1_s, steps, ws, h)
        sims.append(s), hs.append(h), wss.append(ws)
    for s in sims:
        st = scfft.OdeStats()
        scfft.scfft_integrate_wait(s.ctx, st)
        assert st.accepted == steps
    torch.cuda.synchronize()
    for a, b in zip(hs, alone):
        assert torch.equal(a, b)


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_autotune_schedule(prec):
    """The autotuner picks one of the two schedules, keeps the warm start, and
    the next call gives what an untuned context gives (both schedules are
    pinned to the oracle)."""
    cfg = CUBE32
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h = to_dev(torch, state(cfg, seed=3), dt)
    a = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=0)
    b = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=0)
    a.rhs_eval(0.01, h)
    b.rhs_eval(0.01, h)
    fx, ms = scfft.scfft_autotune(b.ctx, h, calls=3)
    assert fx in (0, 2) and ms > 0.0
    oa, _ = a.rhs_eval(0.011, h)                  # second call: from the warm start
    ob, _ = b.rhs_eval(0.011, h)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    assert rel_max(ob.double().cpu().numpy(), oa.double().cpu().numpy()) < tol
    s0 = sim(cfg, precision=prec)                 # adaptive iteration: refused
    with pytest.raises(scfft.ScfftError):
        scfft.scfft_autotune(s0.ctx, h)


def test_graph_reuse_across_calls_and_state_changes():
    """Consecutive graph integrations with the same workspace, step count and
    step size replay the graphs of the first; after a state change (here the
    rhs options: another exterior iteration count) the graphs are captured
    again.  Every result equals the plain fixed-step integrator's."""
    cfg = CUBE32
    dt = torch.float64
    h0 = to_dev(torch, state(cfg, seed=5, bg=(0.0, 0.01, 0.02)), dt)
    steps, chunk = 3, 0.005
    g = sim(cfg, fixed_iter=2)
    p = sim(cfg, fixed_iter=2)
    ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(g.ctx, steps))
    hg, hp = h0.clone(), h0.clone()
    o = scfft.default_ode_opts(fixed_steps=steps)
    for k in range(3):                                    # the same chunk length three times
        t0, t1 = k * chunk, (k + 1) * chunk
        scfft.scfft_integrate_graph(g.ctx, t0, t1, steps, ws, hg)
        scfft.scfft_integrate_wait(g.ctx, scfft.OdeStats())
        scfft.scfft_integrate(p.ctx, t0, t1, hp, o)
        torch.cuda.synchronize()
        assert rel_max(hg.cpu().numpy(), hp.cpu().numpy()) < 1e-12, k
    for s_ in (g, p):
        scfft.scfft_set_rhs_opts(s_.ctx, scfft.default_rhs_opts(fixed_iter=3))
    scfft.scfft_integrate_graph(g.ctx, 3 * chunk, 4 * chunk, steps, ws, hg)
    st = scfft.OdeStats()
    scfft.scfft_integrate_wait(g.ctx, st)
    sp = scfft.OdeStats()
    scfft.scfft_integrate(p.ctx, 3 * chunk, 4 * chunk, hp, o, stats=sp)
    torch.cuda.synchronize()
    assert rel_max(hg.cpu().numpy(), hp.cpu().numpy()) < 1e-12
    assert st.iters_total == sp.iters_total == sp.rhs_calls * 3


@pytest.mark.parametrize("prec,fuse", [(scfft.F64, 0), (scfft.F64, 2), (scfft.F32, 1)])
def test_graph_moment_history(prec, fuse):
    """The moment of every accepted state, summed on the device during graph
    replay, equals what an observer of the plain fixed-step integrator reads
    with scfft_step_moment (all nodes and Omega only)."""
    cfg = CUBE32
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    _, u = oracle_problem(cfg)
    x = np.arange(32) - 15.5
    win = np.exp(-(x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2) / 60.0)
    h0 = to_dev(torch, state(cfg, seed=7) * win, dt)
    t1_s, steps = 0.02, 5
    a = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=fuse)
    ms = []
    scfft.scfft_integrate(a.ctx, 0.0, t1_s, h0.clone(), scfft.default_ode_opts(fixed_steps=steps),
                          observer=lambda _u, t, _p: ms.append((scfft.scfft_step_moment(a.ctx, 0),
                                                                scfft.scfft_step_moment(a.ctx, 1))) or 0)
    b = sim(cfg, precision=prec, fixed_iter=2, fuse_xy=fuse)
    _graph_run(b, h0.clone(), t1_s, steps)
    m_all = scfft.scfft_graph_moments(b.ctx, steps + 3)
    m_in = scfft.scfft_graph_moments(b.ctx, steps, omega_only=1)
    assert m_all.shape == (steps, 3) and m_in.shape == (steps, 3)
    ref_all = np.array([m[0] for m in ms])
    ref_in = np.array([m[1] for m in ms])
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    assert np.max(np.abs(m_all - ref_all)) <= tol * np.max(np.abs(ref_all))
    assert np.max(np.abs(m_in - ref_in)) <= tol * np.max(np.abs(ref_in))
