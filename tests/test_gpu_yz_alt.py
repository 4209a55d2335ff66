"""The alternate element counts of the y passes and of the z passes with the
operator symbols (rhs options y_alt, z_alt: other radix sequences, column
widths and register budgets; schedules the autotuner times): the right-hand
side against the oracle on power-of-two and 3 * 2^k grids, with the row/
column and the fused plane schedules (FP64 <= 1e-10 relative to the largest
reference value, FP32 <= 1e-4 relative L2), and against the default
variants at the full 128^3 size (the variants differ only in rounding
order)."""
import numpy as np
import pytest

from gpu_case import oracle_problem, rel_l2, rel_max, sim, small_cfg, state, to_dev
from oracle import operators
from oracle import rhs as orhs
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TINY = small_cfg((8, 8, 8), (1.0, 1.0, 1.0), workloads.shape_cube(0.5))
NONCUBIC = small_cfg((16, 32, 64), (1.5, 2.0, 3.0), workloads.shape_cup(1.0, 0.6, 3.0, 0.4, axis=1))
CUP64 = workloads.config("cup64")
C48 = small_cfg((48, 96, 24), (2.0, 3.0, 1.2), workloads.shape_cylinder(0.8, 1.6, axis=0))
Z192 = small_cfg((16, 24, 192), (1.0, 1.0, 4.0), workloads.shape_cylinder(0.5, 4.0, axis=2))
Z512 = small_cfg((8, 8, 512), (1.0, 1.0, 8.0), workloads.shape_cylinder(0.5, 6.0, axis=2))
ALTS = [(1, 0), (0, 1), (1, 1)]


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("yz", ALTS, ids=["y", "z", "yz"])
@pytest.mark.parametrize("cfg", [TINY, NONCUBIC, CUP64, C48, Z192, Z512],
                         ids=["8", "16x32x64", "64", "48x96x24", "16x24x192", "8x8x512"])
def test_rhs_yz_alt_fp64(cfg, yz):
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=21)
    dh = to_dev(torch, h, torch.float64)
    want = [orhs.rhs_eval(prob, t_s / u.t0, h) for t_s in (0.25, 0.3)]
    for fuse in (0, 2):
        s = sim(cfg, fixed_iter=3, fuse_xy=fuse, y_alt=yz[0], z_alt=yz[1])
        for t_s, w in zip((0.25, 0.3), want):             # second call uses the warm start
            out, _ = s.rhs_eval(t_s, dh)
            torch.cuda.synchronize()
            assert rel_max(_np(out), w) < 1e-10, (fuse, t_s)
        s.close()


@pytest.mark.parametrize("yz", ALTS, ids=["y", "z", "yz"])
def test_rhs_yz_alt_fp32(yz):
    cfg = C48
    s = sim(cfg, precision=scfft.F32, fixed_iter=3, fuse_xy=0, y_alt=yz[0], z_alt=yz[1])
    prob, u = oracle_problem(cfg, fixed_iter=3)
    h = state(cfg, seed=22)
    out, _ = s.rhs_eval(0.004, to_dev(torch, h, torch.float32))
    torch.cuda.synchronize()
    want = orhs.rhs_eval(prob, 0.004 / u.t0, h)
    assert rel_l2(_np(out), want) < 1e-4


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_yz_alt_matches_default_at_128(prec):
    cfg = workloads.config("cup128")
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    h = to_dev(torch, state(cfg, seed=23), dt)
    outs = []
    for yz in [(0, 0)] + ALTS:
        s = sim(cfg, precision=prec, fixed_iter=3, fuse_xy=0, y_alt=yz[0], z_alt=yz[1])
        o, _ = s.rhs_eval(0.002, h)
        outs.append(_np(o))
        s.close()
    tol = 1e-12 if prec == scfft.F64 else 1e-5
    for o in outs[1:]:
        assert rel_max(o, outs[0]) < tol


def test_autotune_crosses_the_variants():
    """The autotuner's choice is one of the schedules it times, reported by
    scfft_get_rhs_opts, and the tuned context still matches the oracle."""
    cfg = CUP64
    h = state(cfg, seed=24)
    dh = to_dev(torch, h, torch.float64)
    s = sim(cfg, fixed_iter=3)
    fx, ms = scfft.scfft_autotune(s.ctx, dh, calls=2)
    o = scfft.scfft_get_rhs_opts(s.ctx)
    assert o.fuse_xy == fx and fx in (0, 2) and ms > 0.0
    assert o.x_alt in (0, 1) and o.y_alt in (0, 1) and o.z_alt in (0, 1)
    if fx == 2:
        assert o.x_alt == 0
    prob, u = oracle_problem(cfg, fixed_iter=3)
    out, _ = s.rhs_eval(0.003, dh)
    torch.cuda.synchronize()
    assert rel_max(_np(out), orhs.rhs_eval(prob, 0.003 / u.t0, h)) < 1e-10


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("zalt", [0, 1], ids=["default", "alt"])
@pytest.mark.parametrize("nz", [64, 128, 256, 512])
def test_z_operators_every_column_shape(nz, zalt, prec):
    """Curl and Phi (Eq. 4, Eq. 7) with z columns of 64 to 512 nodes in both
    element counts of the Z pass: every shape its column transform takes
    (lane-swapped index bits with one, two or no swaps after the exchange, 8
    or 16 columns per wavefront, or the Stockham passes at 512 nodes with 4
    elements per lane), on full-band random input, against the oracle."""
    n = (16, 16, nz)
    cfg = small_cfg(n, tuple(0.25 * v / 16 for v in n), workloads.shape_cube(0.1))
    s = sim(cfg, precision=prec, z_alt=zalt)
    prob, _ = oracle_problem(cfg)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    dv = to_dev(torch, np.random.default_rng(7 + nz).normal(size=s.field_shape), dt)
    vv = _np(dv)
    out = s.empty_field()
    for op, ref in ((scfft.scfft_curl, operators.curl_s), (scfft.scfft_phi, operators.phi)):
        op(s.ctx, dv, out)
        torch.cuda.synchronize()
        want = ref(vv, prob.grid)
        if prec == scfft.F64:
            assert rel_max(_np(out), want) < 1e-12, (op.__name__, nz, zalt)
        else:
            assert rel_l2(_np(out), want) < 1e-5, (op.__name__, nz, zalt)
    s.close()
