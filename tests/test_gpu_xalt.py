"""The alternate element count of the per-component x passes (rhs option
x_alt = 1, one of the schedules the autotuner times): the right-hand side
against the oracle on power-of-two and 3 * 2^k grids (FP64 <= 1e-10 relative
to the largest reference value, FP32 <= 1e-4 relative L2), with fixed and
adaptive exterior iterations, and against the default schedule at the full
128^3 size (FP64 <= 1e-12, the two differ only in rounding order)."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TINY = small_cfg((8, 8, 8), (1.0, 1.0, 1.0), workloads.shape_cube(0.5))
NONCUBIC = small_cfg((16, 32, 64), (1.5, 2.0, 3.0), workloads.shape_cup(1.0, 0.6, 3.0, 0.4, axis=1))
FLAT = small_cfg((64, 16, 8), (4.0, 1.0, 1.0), workloads.shape_cylinder(0.6, 1.2, axis=0))
CUBE32 = workloads.config("cube32")
CUP64 = workloads.config("cup64")
C48 = small_cfg((48, 32, 24), (2.0, 1.5, 1.2), workloads.shape_cylinder(0.8, 1.6, axis=0))
X192 = small_cfg((192, 24, 24), (4.0, 1.0, 1.0), workloads.shape_cylinder(0.5, 4.0, axis=0))
X128 = small_cfg((128, 16, 16), (4.0, 1.0, 1.0), workloads.shape_cylinder(0.5, 3.0, axis=0))


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("cfg", [TINY, NONCUBIC, FLAT, CUBE32, CUP64, C48, X192, X128],
                         ids=["8", "16x32x64", "64x16x8", "32", "64", "48x32x24", "192x24x24", "128x16x16"])
def test_rhs_x_alt_fp64(cfg):
    s = sim(cfg, fixed_iter=3, fuse_xy=0, x_alt=1)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=12)
    dh = to_dev(torch, h, torch.float64)
    for t_s in (0.25, 0.3):                            # second call uses the warm start
        out, _ = s.rhs_eval(t_s, dh)
        torch.cuda.synchronize()
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        assert rel_max(_np(out), want) < 1e-10, t_s


@pytest.mark.parametrize("cfg", [CUP64, X192], ids=["64", "192x24x24"])
def test_rhs_x_alt_fp32(cfg):
    s = sim(cfg, precision=scfft.F32, fixed_iter=3, fuse_xy=0, x_alt=1)
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=13)
    out, _ = s.rhs_eval(0.004, to_dev(torch, h, torch.float32))
    torch.cuda.synchronize()
    want = orhs.rhs_eval(prob, 0.004 / u.t0, h)
    assert rel_l2(_np(out), want) < 1e-4


def test_rhs_x_alt_adaptive_fp64():
    """Adaptive exterior iteration (the last-iteration and stop-flag passes
    under the alternate count): same iteration count and result as the oracle."""
    cfg = NONCUBIC
    s = sim(cfg, delta_it=2e-5, fuse_xy=0, x_alt=1)
    prob, u = oracle_problem(cfg, delta_it=2e-5)
    h = state(cfg, seed=14)
    dh = to_dev(torch, h, torch.float64)
    for t_s in (0.2, 0.21, 0.22):
        stats = scfft.RhsStats()
        out, _ = s.rhs_eval(t_s, dh, stats=stats)
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        assert stats.iters == prob.last_iters
        assert rel_max(_np(out), want) < 1e-10


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_x_alt_matches_default_at_128(prec):
    cfg = workloads.config("cup128")
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h = to_dev(torch, state(cfg, seed=15), dt)
    outs = []
    for alt in (0, 1):
        s = sim(cfg, precision=prec, fixed_iter=3, fuse_xy=0, x_alt=alt)
        o, _ = s.rhs_eval(0.002, h)
        outs.append(_np(o))
        del s
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    assert rel_max(outs[1], outs[0]) < tol


def test_autotune_reports_its_choice():
    """scfft_get_rhs_opts returns the pair the autotuner kept."""
    cfg = CUBE32
    h = to_dev(torch, state(cfg, seed=16), torch.float64)
    s = sim(cfg, fixed_iter=2, fuse_xy=0)
    s.rhs_eval(0.01, h)
    fx, ms = scfft.scfft_autotune(s.ctx, h, calls=3)
    o = scfft.scfft_get_rhs_opts(s.ctx)
    assert o.fuse_xy == fx and o.x_alt in (0, 1) and ms > 0.0
    if fx == 2:
        assert o.x_alt == 0
