"""Per-kernel timing (scfft_profile / scfft_profile_read): the launch counts
of one right-hand side follow its pass schedule (Sec. 2: 2 + 2k operator
applications), every launch has a positive duration and byte count, the
full-size byte counts follow the per-pass model, and disabling stops the
counting."""
import pytest

from gpu_case import sim, state, to_dev
from paper_1803_01346_amd import scfft, workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_profile_counts_follow_the_schedule():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    cfg = dict(workloads.config("cube32"), n_power=20.0)
    K, calls = 3, 4
    s = sim(cfg, fixed_iter=K, fuse_xy=0, prune_box=0)
    h = to_dev(torch, state(cfg, seed=1), torch.float64)
    hd = s.empty_field()
    s.rhs_eval(0.01, h, hd)                                  # warm start exists from here on
    scfft.scfft_profile(s.ctx, 1)
    for _ in range(calls):
        s.rhs_eval(0.01, h, hd)
    prof = scfft.scfft_profile_read(s.ctx)
    scfft.scfft_profile(s.ctx, 0)
    n_ops = 2 + 2 * K                                        # spectral operator applications
    want = {"X_FWD": 1, "X_LAW": 1, "X_HIN": 1, "X_MASK": K, "X_UPDATE": K - 1, "X_UPDATE_LAST": 1,
            "Y_FWD": n_ops, "Y_INV": n_ops, "Z_CURL": 2 + K, "Z_PHI": K}
    for kind, per_call in want.items():
        la, ms, by = prof[kind]
        assert la == per_call * calls, kind
        assert ms > 0.0 and by > 0.0, kind
    assert all(prof[k][0] == 0 for k in prof if k not in want)
    # full transforms (no pruning): a Y or Z pass reads and writes the half spectrum
    n = cfg["n"]
    S = 3 * n[2] * n[1] * (n[0] // 2) * 16
    assert prof["Y_FWD"][2] / prof["Y_FWD"][0] == pytest.approx(2 * S)
    assert prof["Z_CURL"][2] / prof["Z_CURL"][0] == pytest.approx(2 * S)
    s.rhs_eval(0.01, h, hd)                                  # not counted once disabled
    assert scfft.scfft_profile_read(s.ctx)["X_FWD"][0] == calls
