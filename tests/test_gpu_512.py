"""The largest grid the library takes, 512^3: the same closed forms as the
256^3 checks (C_s of a separable field with random profiles, exact at every
node; Phi of a sum of Fourier modes, Eq. 7), in FP64 and FP32.  One field
component is 1 GiB in FP64 here, so the passes' array sizes and 32-bit load
offsets reach their largest values, and the z columns of 512 nodes take both
forms of the column transform (Stockham passes with 4 elements per lane in
FP64, the lane-swapped form with 8 in FP32)."""
import numpy as np
import pytest

from gpu_case import rel_max, sim, small_cfg, to_dev
from oracle import grid as ogrid
from paper_1803_01346_amd import scfft, workloads
from test_gpu_256 import _separable_curl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BIG = small_cfg((512, 512, 512), (1.0, 1.0, 1.0), workloads.shape_cube(0.3))


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_curl_separable_512(prec):
    g = ogrid.Grid(BIG["n"], BIG["half_width"])
    rng = np.random.default_rng(41)
    prof = [[rng.normal(size=n) for n in g.n] for _ in range(3)]
    v = np.stack([p[2][:, None, None] * p[1][None, :, None] * p[0][None, None, :] for p in prof])
    want = _separable_curl(prof, g)
    s = sim(BIG, precision=prec)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    dv = to_dev(torch, v, dt)
    del v
    out = s.empty_field()
    scfft.scfft_curl(s.ctx, dv, out)
    torch.cuda.synchronize()
    err = rel_max(_np(out), want)
    s.close()
    assert err < (1e-12 if prec == scfft.F64 else 2e-5), err


@pytest.mark.parametrize("prec", [scfft.F64, scfft.F32], ids=["f64", "f32"])
def test_phi_modes_512(prec):
    g = ogrid.Grid(BIG["n"], BIG["half_width"])
    x, y, z = g.mesh_nodes()
    rng = np.random.default_rng(42)
    j = np.zeros((3,) + g.shape)
    want = np.zeros((3,) + g.shape)
    for _ in range(4):
        m = rng.integers(-g.n[0] // 8, g.n[0] // 8 + 1, size=3)
        if not m.any():
            m[2] = 1
        k = np.pi * m / np.asarray(g.L)
        a = rng.normal(size=3)
        th = k[0] * x + k[1] * y + k[2] * z + rng.uniform(0.0, 2.0 * np.pi)
        c, sn = np.cos(th), np.sin(th)
        del th
        kxa = np.cross(k, a) / float(k @ k)
        for comp in range(3):
            j[comp] += a[comp] * c
            want[comp] -= kxa[comp] * sn
        del c, sn
    del x, y, z
    s = sim(BIG, precision=prec)
    dt = torch.float64 if prec == scfft.F64 else torch.float32
    dj = to_dev(torch, j, dt)
    del j
    out = s.empty_field()
    scfft.scfft_phi(s.ctx, dj, out)
    torch.cuda.synchronize()
    err = rel_max(_np(out), want)
    s.close()
    assert err < (1e-12 if prec == scfft.F64 else 2e-5), err
