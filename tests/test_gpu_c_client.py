"""A plain C program (tests/c/cube_ramp.c) driving the library through the C
ABI alone gives what the Python binding gives for the same run: the cube
under a 0.1 T ramp, adaptive steps from the virgin state, moment at 1 s and
2 s."""
import os
import subprocess

import numpy as np
import pytest

from paper_1803_01346_amd import scfft, workloads
from test_abi import _build_c_client

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_c_client_matches_python(tmp_path):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    exe = _build_c_client(str(tmp_path / "cube_ramp"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = [dict(zip(l.split()[0::2], l.split()[1::2])) for l in r.stdout.strip().splitlines()]
    assert len(rows) == 2
    cfg = dict(workloads.config("cube32"))
    s = scfft.Simulation(cfg, precision=scfft.F64)
    h = s.empty_field()
    scfft.scfft_init_state(s.ctx, 0.0, h)
    t = 0.0
    for row, t1 in zip(rows, (1.0, 2.0)):
        st = scfft.OdeStats()
        scfft.scfft_integrate(s.ctx, t, t1, h, scfft.default_ode_opts(), stats=st)
        m = scfft.scfft_moment(s.ctx, h, 0)
        assert int(row["accepted"]) == st.accepted and int(row["rhs"]) == st.rhs_calls
        assert abs(float(row["m_z"]) - m[2]) <= 1e-12 * abs(m[2])
        t = t1
