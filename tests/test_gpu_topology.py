"""The context's topology warning: voxelizing or setting a mask that is not
contourwise simply connected (Sec. 2) returns the warning status, keeps the
mask, and the Python layer turns it into a warning."""
import warnings

import numpy as np
import pytest

from gpu_case import small_cfg
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LENS = workloads.shape_lens(1.0, 4.0 / 3.0, 0.2, 0.15)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    scfft.load()


def test_topology_warning_on_context():
    ring = small_cfg((32, 32, 32), (1.2, 1.2, 1.2), LENS[:2])
    with pytest.warns(UserWarning, match="simply connected"):
        s = scfft.Simulation(ring, precision=scfft.F64)
    assert scfft.scfft_mask_betti(s.ctx) == (1, 1, 0)
    ok = small_cfg((32, 32, 32), (1.2, 1.2, 1.2), LENS)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        s2 = scfft.Simulation(ok, precision=scfft.F64)
    assert scfft.scfft_mask_betti(s2.ctx) == (1, 0, 0)
    # a device mask: the ring's voxels, then the slit lens's again
    ring_mask = np.zeros((32, 32, 32), np.uint8)
    ring_mask[12:20, 8:24, 8:24] = 1
    ring_mask[12:20, 12:20, 12:20] = 0
    st = scfft.scfft_set_mask(s2.ctx, torch.from_numpy(ring_mask).cuda())
    assert st == scfft.WARN_TOPOLOGY and scfft.scfft_mask_betti(s2.ctx) == (1, 1, 0)
    out, _ = s2.rhs_eval(0.0, s2.empty_field().zero_())   # the mask is in use
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
