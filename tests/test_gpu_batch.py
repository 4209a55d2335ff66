"""Batches of same-size instances (scfft_batch_*): one launch per pass over
all members, instance = blockIdx.z.

* Every instance of a mixed batch (box edges 48 to 192, bodies, n, jc and
  field directions drawn by workloads.batch_instances) gets, bit for bit,
  the right-hand side its own context gives alone, first and warm-started
  call: the batched launches run the same arithmetic per instance.
* The instances of edge 48, 64 and 96 against the FP64 oracle (<= 1e-10
  relative max); the single-context path at 128^3 is checked against the
  oracle on all nodes in test_gpu_parity.py, and the oracle's direct DFT
  makes 192^3 unaffordable.
* The graph-replayed batched integration equals each member's own
  graph-replayed integration bit for bit.
* Members that do not fit together are refused.
"""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_max, to_dev
from oracle import rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIXED = 3


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


def _np(t):
    return t.detach().double().cpu().numpy()


def _by_edge(per_edge=3):
    """Instances of the seeded mixed batch, up to per_edge of each box edge."""
    groups = {}
    for c in workloads.batch_instances(64):
        groups.setdefault(c["n"][0], [])
        if len(groups[c["n"][0]]) < per_edge:
            groups[c["n"][0]].append(c)
    return groups


def _states(cfgs, seed0=0):
    return [workloads.synthetic_state(c, seed=seed0 + i, background=(0.0, 0.0, 0.0)) for i, c in enumerate(cfgs)]


def _opts():
    return scfft.default_rhs_opts(fixed_iter=FIXED)


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_batch_rhs_equals_single_contexts_bitwise(prec):
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    for edge, cfgs in sorted(_by_edge().items()):
        hs = _states(cfgs)
        b = scfft.Batch(cfgs, precision=prec, rhs_opts=_opts())
        h = torch.stack([to_dev(torch, x, dt) for x in hs]).contiguous()
        singles = [scfft.Simulation(c, precision=prec, rhs_opts=_opts()) for c in cfgs]
        for t_s in (0.2, 0.21):                                     # second call: warm start
            got = b.rhs_eval(t_s, h)
            want = [s.rhs_eval(t_s, h[i])[0] for i, s in enumerate(singles)]
            torch.cuda.synchronize()
            for i, w in enumerate(want):
                assert torch.equal(got[i], w), (edge, i, t_s)
        b.close()
        for s in singles:
            s.close()


def test_batch_rhs_against_oracle():
    groups = _by_edge(per_edge=2)
    for edge in (48, 64, 96):
        cfgs = groups[edge][:2] if edge < 96 else groups[edge][:1]
        hs = _states(cfgs, seed0=10)
        b = scfft.Batch(cfgs, precision=scfft.F64, rhs_opts=_opts())
        h = torch.stack([to_dev(torch, x, torch.float64) for x in hs]).contiguous()
        probs = [oracle_problem(c, fixed_iter=FIXED) for c in cfgs]
        for t_s in (0.2, 0.21):
            got = _np(b.rhs_eval(t_s, h))
            for i, (prob, u) in enumerate(probs):
                want = orhs.rhs_eval(prob, t_s / u.t0, hs[i])
                err = rel_max(got[i], want)
                print("batch edge %d instance %d t=%g: rel max %.2e" % (edge, i, t_s, err))
                assert err < 1e-10, (edge, i, t_s)
        b.close()


def test_batch_rhs_against_oracle_128():
    """Two 128^3 members of the mixed set in one batched call against the
    oracle (about 15 s per oracle call; the 3 * 2^k edges are compared at 96,
    where the oracle's transform is affordable: at 192^3 it takes minutes)."""
    edge, count = 128, 2
    cfgs = _by_edge(per_edge=count)[edge][:count]
    hs = _states(cfgs, seed0=30)
    b = scfft.Batch(cfgs, precision=scfft.F64, rhs_opts=_opts())
    h = torch.stack([to_dev(torch, x, torch.float64) for x in hs]).contiguous()
    got = _np(b.rhs_eval(0.2, h))
    b.close()
    for i, c in enumerate(cfgs):
        prob, u = oracle_problem(c, fixed_iter=FIXED)
        want = orhs.rhs_eval(prob, 0.2 / u.t0, hs[i])
        err = rel_max(got[i], want)
        print("batch edge %d instance %d: rel max %.2e" % (edge, i, err))
        assert err < 1e-10, (edge, i)


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_batch_graph_equals_single_graphs(prec):
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    cfgs = _by_edge(per_edge=4)[48]
    hs = _states(cfgs, seed0=20)
    steps, t1 = 3, 2e-4
    b = scfft.Batch(cfgs, precision=prec, rhs_opts=_opts())
    h = torch.stack([to_dev(torch, x, dt) for x in hs]).contiguous()
    b.integrate_graph(0.0, t1, steps, h)
    st = b.wait()
    assert [s.accepted for s in st] == [steps] * len(cfgs)
    for i, c in enumerate(cfgs):
        s = scfft.Simulation(c, precision=prec, rhs_opts=_opts())
        hi = to_dev(torch, hs[i], dt)
        ws = scfft.device_buffer(scfft.scfft_graph_workspace_size(s.ctx, steps))
        scfft.scfft_integrate_graph(s.ctx, 0.0, t1, steps, ws, hi)
        so = scfft.OdeStats()
        scfft.scfft_integrate_wait(s.ctx, so)
        torch.cuda.synchronize()
        assert torch.equal(h[i], hi), i
        assert st[i].err_last == so.err_last and st[i].rhs_calls == so.rhs_calls
        s.close()
    b.close()


def test_batch_members_must_fit():
    cfgs = _by_edge(per_edge=2)
    a = scfft.Simulation(cfgs[48][0], rhs_opts=_opts())
    c = scfft.Simulation(cfgs[64][0], rhs_opts=_opts())
    with pytest.raises(scfft.ScfftError) as e:                  # other grid
        scfft.scfft_batch_create([a.ctx, c.ctx])
    assert e.value.status == scfft.ERR_SHAPE
    d = scfft.Simulation(cfgs[48][1], rhs_opts=_opts())
    with pytest.raises(scfft.ScfftError) as e:                  # a member twice
        scfft.scfft_batch_create([a.ctx, d.ctx, a.ctx])
    assert e.value.status == scfft.ERR_ARG
    f = scfft.Simulation(cfgs[48][1], rhs_opts=scfft.default_rhs_opts(fixed_iter=0))
    with pytest.raises(scfft.ScfftError):                       # the stopping rule is per call
        scfft.scfft_batch_create([a.ctx, f.ctx])
    for s in (a, c, d, f):
        s.close()
