"""Pins of the scaling of Eq. 8 and the drives, against numbers the paper
prints (tests/golden/paper_constants.json)."""
import json
import os

import numpy as np

from oracle import units

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_lens_example_fields():
    # Sec. 3: OD 30 mm, jc = 5e8 A/m^2; |h_e| = 0.05 and 0.2 <-> 0.473 T and 1.89 T.
    ex = GOLD["lens_unit_example"]
    u = units.Units(ex["jc_A_per_m2"], 0.5 * ex["outer_diameter_m"])
    for pair in ex["pairs"]:
        b = float(u.field_dimless_to_T(pair["h_dimless"]))
        assert abs(b - pair["B_T"]) / pair["B_T"] < 5e-3      # printed to 3 digits
        assert abs(float(u.field_T_to_dimless(b)) - pair["h_dimless"]) < 1e-15
    # the characteristic length these figures imply is the outer radius (to 0.4 %)
    l_implied = ex["pairs"][0]["B_T"] / (ex["pairs"][0]["h_dimless"] * units.MU0 * ex["jc_A_per_m2"])
    assert abs(l_implied / (0.5 * ex["outer_diameter_m"]) - 1.0) < 5e-3


def test_time_scale_definition():
    u = units.Units(1e8, 5e-3)
    # t0 = mu0 jc l^2 / e0 with e0 = 1e-4 V/m (the paper's e0)
    assert GOLD["e0_V_per_m"]["value"] == units.E0_DEFAULT
    assert np.isclose(u.t0, 4e-7 * np.pi * 1e8 * 25e-6 / 1e-4, rtol=1e-15)
    assert np.isclose(u.t0, 31.41592653589793, rtol=1e-14)


def test_drives():
    u = units.Units(1e8, 5e-3)
    r = units.Drive(u, "ramp_hold", (0, 0, 2.0), 0.1, 1.0)
    tr = 1.0 / u.t0
    amp = 0.1 / units.MU0 / (1e8 * 5e-3)
    assert np.allclose(r.he(0.5 * tr), [0, 0, 0.5 * amp]) and np.allclose(r.he(3 * tr), [0, 0, amp])
    assert np.allclose(r.hedot(0.5 * tr), [0, 0, amp / tr]) and np.all(r.hedot(2 * tr) == 0)
    assert r.breakpoints() == [tr]
    s = units.Drive(u, "sine", (1, 0, 1), 0.05, freq_hz=50.0)
    t = 0.003 / u.t0
    a = 0.05 / units.MU0 / (1e8 * 5e-3)
    w = 2 * np.pi * 50 * u.t0
    assert np.allclose(s.he(t), np.sqrt(0.5) * a * np.sin(w * t) * np.array([1, 0, 1]))
    eps = 1e-6 * t
    fd = (s.he(t + eps) - s.he(t - eps)) / (2 * eps)
    assert np.allclose(s.hedot(t), fd, rtol=1e-6)
    p = units.Drive(u, "pwl", t_s=[0.0, 1.0, 2.0], b_T=[[0, 0, 0], [0, 0, 0.1], [0.1, 0, 0.1]])
    assert np.allclose(p.he(1.5 / u.t0), [0.5 * amp, 0, amp])
    assert np.allclose(p.hedot(1.5 / u.t0), [amp / tr, 0, 0])
