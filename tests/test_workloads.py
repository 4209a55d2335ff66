"""The seeded input generators: the device-side synthetic state equals the
host one (same modes from the same generator), and the batch instances have
the mixed sizes they promise."""
import numpy as np

from paper_1803_01346_amd import workloads


def test_torch_state_equals_numpy_state():
    cfg = dict(workloads.config("cube32"), n=(16, 24, 32))
    a = workloads.synthetic_state(cfg, seed=5, background=(0.1, 0.0, -0.2))
    b = workloads.synthetic_state_torch(cfg, seed=5, background=(0.1, 0.0, -0.2), device="cpu").numpy()
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_batch_instances_mix_sizes():
    b = workloads.batch_instances()
    assert len(b) == 64
    edges = {c["n"][0] for c in b}
    assert edges == {48, 64, 96, 128, 192}
    assert all(c["n"][0] == c["n"][1] == c["n"][2] for c in b)
    assert all(10.0 <= c["n_power"] <= 100.0 and 1e7 <= c["jc"] <= 1e9 for c in b)
