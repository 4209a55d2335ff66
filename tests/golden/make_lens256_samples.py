"""Write lens256_rhs_samples.npz: the FP64 oracle's right-hand side of the
256^3 lens box sampled at chosen nodes (test infrastructure only).

The oracle's full 3D transforms at 256^3 take minutes, so the GPU parity
test at that size compares sampled nodes against values this script stores.
It calls only oracle/ (and the seeded input generator of the workloads
module, which holds no arithmetic of the method).

Workload: the slit lens on the 256^3 box (n = 50, rho_out = 100, jc = 2e8
A/m^2, l = 15 mm), state = synthetic_state(seed 0) on a 0.1 background along
the axis, 3 exterior iterations (Eq. 5) per call; two calls in a row at
t = 10 s (Ohm-law start, Sec. 2) and t = 10.5 s (warm start from the first).

Samples: 8192 nodes drawn with numpy.random.default_rng(256), the four node
columns straddling the bore axis, and the x and y node lines through the box
centre (the x line crosses the slit).  Stored per call: the values at the
samples, the largest magnitude over all nodes and components (the rel-max
normaliser) and, as a guard against drift of the input generator, the
SHA-256 of the input h at the samples (float64, C order).

    python tests/golden/make_lens256_samples.py      # about 20 minutes
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import geometry, grid, rhs, units  # noqa: E402
from paper_1803_01346_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "lens256_rhs_samples.npz")
T_S = (10.0, 10.5)
FIXED_ITER = 3
SEED_STATE = 0
SEED_SAMPLES = 256
BACKGROUND = (0.0, 0.0, 0.1)


def sample_nodes(n):
    nx, ny, nz = n
    rng = np.random.default_rng(SEED_SAMPLES)
    rand = rng.choice(nx * ny * nz, size=8192, replace=False)
    zc, yc, xc = nz // 2, ny // 2, nx // 2
    axis = [(z * ny + y) * nx + x for z in range(nz) for y in (yc - 1, yc) for x in (xc - 1, xc)]
    xline = [(zc * ny + yc) * nx + x for x in range(nx)]
    yline = [(zc * ny + y) * nx + xc for y in range(ny)]
    return np.unique(np.concatenate([rand, axis, xline, yline]).astype(np.int64))


def input_digest(h_at):
    return hashlib.sha256(np.ascontiguousarray(h_at, dtype=np.float64).tobytes()).hexdigest()


def main():
    cfg = workloads.config("lens256")
    g = grid.Grid(cfg["n"], cfg["half_width"])
    chi = geometry.voxelize(g, cfg["shapes"])
    u = units.Units(cfg["jc"], cfg["l_m"], cfg["e0"])
    d = dict(cfg["drive"])
    drive = units.Drive(u, d.pop("kind"), **d)
    prob = rhs.Problem(g, chi, cfg["n_power"], cfg["rho_out"], drive,
                       rhs.RhsOptions(fixed_iter=FIXED_ITER))
    h = workloads.synthetic_state(cfg, seed=SEED_STATE, background=BACKGROUND)
    idx = sample_nodes(cfg["n"])
    flat = h.reshape(3, -1)
    out = dict(idx=idx, t_s=np.array(T_S), fixed_iter=FIXED_ITER, seed_state=SEED_STATE,
               background=np.array(BACKGROUND), chi_at=chi.reshape(-1)[idx],
               h_sha256=np.array(input_digest(flat[:, idx])))
    for k, t_s in enumerate(T_S):
        t = time.perf_counter()
        hdot = rhs.rhs_eval(prob, t_s / u.t0, h)
        f = hdot.reshape(3, -1)
        out["hdot%d" % k] = f[:, idx]
        out["scale%d" % k] = float(np.max(np.abs(f)))
        out["l2_%d" % k] = float(np.sqrt(np.sum(f * f)))
        print("call %d (t = %g s): %.0f s, max |hdot| %.6g" % (k, t_s, time.perf_counter() - t,
                                                               out["scale%d" % k]), flush=True)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT, "with", idx.size, "sampled nodes")


if __name__ == "__main__":
    main()
