"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side logic (voxelizer, drives, scaling, step controller)
agrees with the oracle.  No device work is done here."""
import math
import os
import re

import numpy as np
import pytest

from oracle import geometry, grid, ode, units
from paper_1803_01346_amd import scfft, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "scfft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scfft_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = scfft.load()
    names = _declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(scfft.exported_symbols())


def test_status_strings():
    for s in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6, -7, -8):
        assert scfft.scfft_status_string(s) != "unknown status"


@pytest.mark.parametrize("name", list(workloads.CONFIGS))
def test_voxelizer_matches_oracle_bitwise(name):
    c = workloads.config(name)
    if c["n"][0] > 128:
        c = dict(c, n=(128, 128, 128))
    g = scfft.make_grid(c["n"], [v * c["l_m"] for v in c["half_width"]])
    m = scfft.make_material(c["n_power"], c["jc"], 1e-4, c["rho_out"], c["l_m"])
    sh, ns = scfft.make_shapes(c["shapes"], c["l_m"])
    lib_mask = scfft.scfft_voxelize_host(g, m, sh, ns)
    orc = geometry.voxelize(grid.Grid(c["n"], c["half_width"]), c["shapes"])
    assert lib_mask.sum() > 0
    assert np.array_equal(lib_mask, orc)


def test_voxelizer_non_cubic_and_sphere():
    shapes = workloads.shape_sphere(0.9) + [workloads.prim("box", "sub", (0.5, 0, 0), (0.2, 0.3, 0.4))]
    n, L, l = (16, 32, 8), (1.0, 1.5, 1.2), 2e-3
    g = scfft.make_grid(n, [v * l for v in L])
    m = scfft.make_material(30, 1e8, 1e-4, 20, l)
    sh, ns = scfft.make_shapes(shapes, l)
    assert np.array_equal(scfft.scfft_voxelize_host(g, m, sh, ns),
                          geometry.voxelize(grid.Grid(n, L), shapes))


def test_units_and_drives_match_oracle():
    m = scfft.make_material(30, 5e8, 1e-4, 20, 0.015)
    t0, hs = scfft.scfft_units(m)
    u = units.Units(5e8, 0.015)
    assert math.isclose(t0, u.t0, rel_tol=1e-15) and math.isclose(hs, u.h_scale, rel_tol=1e-15)
    cases = [dict(kind="ramp_hold", direction=(0, 1, 1), amp_T=0.3, t_ramp_s=2.0),
             dict(kind="sine", direction=(1, 0, 1), amp_T=0.05, freq_hz=50.0),
             dict(kind="pwl", t_s=[0.0, 1.0, 3.0], b_T=[[0, 0, 0], [0, 0, 0.1], [0.1, 0, 0.1]])]
    for d in cases:
        dd = dict(d)
        kind = dd.pop("kind")
        lib_d = scfft.make_drive(kind, **dd)
        orc = units.Drive(u, kind, **{k: v for k, v in dd.items()})
        for t_s in (0.0, 0.2, 1.0, 1.7, 2.5, 5.0):
            he, hd = scfft.scfft_drive_eval(lib_d, m, t_s)
            tt = t_s / u.t0
            assert np.allclose(he, orc.he(tt), rtol=1e-14, atol=1e-300)
            assert np.allclose(hd, orc.hedot(tt), rtol=1e-14, atol=1e-300)


def test_host_bs23_matches_oracle_controller():
    f = lambda t, y: np.array([y[0] * np.cos(t) + 0.1 * np.sin(3 * t), -0.5 * y[1]])
    o = scfft.default_ode_opts(rtol=1e-5, atol=1e-8, breakpoints_s=[0.7])
    rc, y, st = scfft.scfft_bs23_host([1.0, 2.0], 0.0, 2.0, f, o)
    yo, so = ode.integrate(f, 0.0, 2.0, np.array([1.0, 2.0]), rtol=1e-5, atol=1e-8, breakpoints=[0.7])
    assert rc == 0
    assert st.accepted == so.accepted and st.rejected == so.rejected
    assert st.rhs_calls == so.rhs_calls
    assert np.allclose(y, yo, rtol=1e-12)


def test_host_bs23_fixed_steps_exact_cubic():
    lam = -2.0
    o = scfft.default_ode_opts(fixed_steps=1)
    rc, y, st = scfft.scfft_bs23_host([1.0], 0.0, 0.1, lambda t, y: lam * y, o)
    z = lam * 0.1
    assert rc == 0 and abs(y[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15
    assert st.rhs_calls == 4


def test_host_bs23_nan_is_reported():
    o = scfft.default_ode_opts()
    rc, y, st = scfft.scfft_bs23_host([1.0], 0.0, 1.0, lambda t, y: np.array([np.nan]), o)
    assert rc == scfft.ERR_NAN


def test_host_bs23_rejects_bad_options():
    o = scfft.default_ode_opts(rtol=-1.0)
    rc, _, _ = scfft.scfft_bs23_host([1.0], 0.0, 1.0, lambda t, y: y, o)
    assert rc == scfft.ERR_ARG


def test_create_rejects_bad_shapes():
    m = scfft.make_material(30, 1e8, 1e-4, 20, 1e-2)
    for n in ((12, 16, 16), (4, 16, 16), (1024, 8, 8)):
        with pytest.raises(scfft.ScfftError) as e:
            scfft.scfft_create(scfft.make_grid(n, (0.01, 0.01, 0.01)), m)
        assert e.value.status == scfft.ERR_SHAPE
    with pytest.raises(scfft.ScfftError) as e:
        scfft.scfft_create(scfft.make_grid((16, 16, 16), (0.01, 0.01, 0.01)),
                           scfft.make_material(0.5, 1e8, 1e-4, 20, 1e-2))
    assert e.value.status == scfft.ERR_ARG


def _build_c_client(out):
    """Compile tests/c/cube_ramp.c, a plain C client of include/scfft.h,
    against the in-tree library with the system C compiler."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pkg = os.path.join(ROOT, "paper_1803_01346_amd")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "cube_ramp.c"), "-L" + pkg, "-lscfft",
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + pkg, "-Wl,-rpath,/opt/rocm/lib", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return out


def test_c_client_compiles_and_links(tmp_path):
    """The header is plain C11 and the library links into a C program."""
    scfft.load()                                       # the library is built
    assert os.path.exists(_build_c_client(str(tmp_path / "cube_ramp")))
