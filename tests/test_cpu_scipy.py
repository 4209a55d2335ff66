"""The multi-core scipy.fft right-hand side that bench.py times as CPU
context equals the oracle's (3 exterior iterations, first and warm-started
call) to round-off, so the context figure is for a correct implementation."""
import numpy as np

from gpu_case import oracle_problem, rel_max, small_cfg, state
from oracle import rhs as orhs
import bench
from paper_1803_01346_amd import workloads


def test_scipy_rhs_matches_oracle():
    cfg = small_cfg((32, 16, 24), (2.0, 1.0, 1.5), workloads.shape_cup(0.8, 0.5, 2.0, 0.3))
    prob, u = oracle_problem(cfg, fixed_iter=3)
    f = bench.ScipyRhs(cfg["n"], cfg["half_width"], prob.chi, cfg["n_power"], cfg["rho_out"], 3,
                           workers=2)
    h = state(cfg, seed=5)
    for t_s in (0.2, 0.21):
        want = orhs.rhs_eval(prob, t_s / u.t0, h)
        got = f(prob.drive.hedot(t_s / u.t0), h)
        assert rel_max(got, want) < 1e-12, t_s
