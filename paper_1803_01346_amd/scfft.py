"""Python binding of libscfft (ctypes).  Argument marshalling only: every
step of the computation runs in the HIP library.  PyTorch supplies device
memory (tensors) and streams.

The functions mirror the C ABI declared in include/scfft.h one to one
(same names, same argument order; host arrays may be numpy arrays or
sequences, device arrays are torch tensors or raw integer addresses).
`Simulation` bundles a context, its workspace tensor and the usual calls.
"""
import ctypes as C
import os
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SCFFT_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SCFFT_LIBRARY") or os.path.join(_HERE, "libscfft.so")

OK = 0
WARN_NOT_CONVERGED = 1
WARN_CLAMPED = 2
WARN_TOPOLOGY = 3
ERR_ARG, ERR_SHAPE, ERR_DEVICE, ERR_WORKSPACE = -1, -2, -3, -4
ERR_NAN, ERR_STEP_UNDERFLOW, ERR_GEOMETRY, ERR_STATE = -5, -6, -7, -8
F64, F32 = 0, 1
DRIVE_RAMP_HOLD, DRIVE_SINE, DRIVE_PWL = 0, 1, 2
SHAPE_BOX, SHAPE_CYLINDER, SHAPE_SPHERE = 0, 1, 2
OP_ADD, OP_SUB = 0, 1


class ScfftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("scfft status %d: %s" % (status, msg))
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("half_width_m", C.c_double * 3)]


class Material(C.Structure):
    _fields_ = [("n_power", C.c_double), ("jc", C.c_double), ("e0", C.c_double),
                ("rho_out", C.c_double), ("l_char_m", C.c_double)]


class Drive(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_pts", C.c_int32), ("dir", C.c_double * 3),
                ("amp_T", C.c_double), ("t_ramp_s", C.c_double), ("freq_hz", C.c_double),
                ("t_s", C.POINTER(C.c_double)), ("b_T", C.POINTER(C.c_double))]


class Shape(C.Structure):
    _fields_ = [("kind", C.c_int32), ("op", C.c_int32), ("axis", C.c_int32),
                ("reserved", C.c_int32), ("center_m", C.c_double * 3), ("size_m", C.c_double * 3)]


class RhsOpts(C.Structure):
    _fields_ = [("delta_it", C.c_double), ("min_iter", C.c_int32), ("max_iter", C.c_int32),
                ("fixed_iter", C.c_int32), ("smooth_phi", C.c_int32), ("sigma_scale", C.c_double),
                ("fuse_xy", C.c_int32), ("prune_box", C.c_int32), ("x_alt", C.c_int32),
                ("y_alt", C.c_int32), ("z_alt", C.c_int32)]


class RhsStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("last_delta", C.c_double),
                ("clamps", C.c_int64)]


class OdeOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("dt0_s", C.c_double),
                ("dt_max_s", C.c_double), ("fixed_steps", C.c_int32), ("n_bp", C.c_int32),
                ("breakpoints_s", C.POINTER(C.c_double)), ("max_steps", C.c_int64),
                ("resume", C.c_int32), ("reserved", C.c_int32)]


class OdeStats(C.Structure):
    _fields_ = [("accepted", C.c_int64), ("rejected", C.c_int64), ("rhs_calls", C.c_int64),
                ("iters_total", C.c_int64), ("not_converged", C.c_int64), ("clamps", C.c_int64),
                ("t_s", C.c_double), ("dt_last_s", C.c_double), ("err_last", C.c_double)]


OBSERVER = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_double, C.c_void_p)
HOST_RHS = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_double, C.POINTER(C.c_double),
                       C.POINTER(C.c_double))

_P = C.c_void_p
_SIGS = {
    "scfft_default_rhs_opts": (None, [C.POINTER(RhsOpts)]),
    "scfft_default_ode_opts": (None, [C.POINTER(OdeOpts)]),
    "scfft_units": (C.c_int, [C.POINTER(Material), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "scfft_drive_eval": (C.c_int, [C.POINTER(Drive), C.POINTER(Material), C.c_double,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "scfft_voxelize_host": (C.c_int, [C.POINTER(Grid), C.POINTER(Material), C.POINTER(Shape),
                                      C.c_int32, C.POINTER(C.c_uint8)]),
    "scfft_bs23_host": (C.c_int, [C.c_int64, C.POINTER(C.c_double), C.c_double, C.c_double,
                                  HOST_RHS, _P, C.POINTER(OdeOpts), C.POINTER(OdeStats)]),
    "scfft_create": (C.c_int, [C.POINTER(_P), C.POINTER(Grid), C.POINTER(Material), C.c_int, _P]),
    "scfft_destroy": (None, [_P]),
    "scfft_workspace_size": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "scfft_set_workspace": (C.c_int, [_P, _P, C.c_size_t]),
    "scfft_voxelize": (C.c_int, [_P, C.POINTER(Shape), C.c_int32]),
    "scfft_set_mask": (C.c_int, [_P, _P]),
    "scfft_mask_betti": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "scfft_stray_fraction": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "scfft_get_rhs_opts": (C.c_int, [_P, _P]),
    "scfft_graph_moments": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int32)]),
    "scfft_mask_betti_host": (C.c_int, [C.POINTER(C.c_int32), C.POINTER(C.c_uint8), C.POINTER(C.c_int64)]),
    "scfft_set_jc_map": (C.c_int, [_P, _P]),
    "scfft_set_drive": (C.c_int, [_P, C.POINTER(Drive)]),
    "scfft_set_field_law": (C.c_int, [_P, C.c_double, C.c_double]),
    "scfft_set_anisotropy": (C.c_int, [_P, _P]),
    "scfft_set_rhs_opts": (C.c_int, [_P, C.POINTER(RhsOpts)]),
    "scfft_reset_warm": (C.c_int, [_P]),
    "scfft_init_state": (C.c_int, [_P, C.c_double, _P]),
    "scfft_rhs_eval": (C.c_int, [_P, C.c_double, _P, _P, C.POINTER(RhsStats)]),
    "scfft_integrate": (C.c_int, [_P, C.c_double, C.c_double, _P, C.POINTER(OdeOpts), OBSERVER,
                                  _P, C.POINTER(OdeStats)]),
    "scfft_curl": (C.c_int, [_P, _P, _P]),
    "scfft_curl_noalloc": (C.c_int, [_P, _P, _P]),
    "scfft_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(_P), C.c_int32]),
    "scfft_batch_destroy": (None, [_P]),
    "scfft_batch_rhs_eval": (C.c_int, [_P, C.c_double, _P, _P, C.c_int64]),
    "scfft_batch_graph_workspace_size": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
    "scfft_batch_integrate_graph": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P, C.c_size_t, _P,
                                              C.c_int64]),
    "scfft_batch_integrate_wait": (C.c_int, [_P, C.POINTER(OdeStats)]),
    "scfft_batch_last_error": (C.c_char_p, [_P]),
    "scfft_phi": (C.c_int, [_P, _P, _P]),
    "scfft_current": (C.c_int, [_P, _P, _P]),
    "scfft_moment": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_double)]),
    "scfft_step_moment": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_double)]),
    "scfft_autotune": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "scfft_graph_workspace_size": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_size_t)]),
    "scfft_integrate_graph": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, _P, C.c_size_t, _P]),
    "scfft_integrate_wait": (C.c_int, [_P, C.POINTER(OdeStats)]),
    "scfft_rhs_vjp": (C.c_int, [_P, _P, C.c_int32, _P, _P, _P, _P, _P, C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
    "scfft_adjoint_workspace_size": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "scfft_integrate_adjoint": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32, C.c_int32, _P,
                                          C.c_size_t, _P, _P, _P, _P, _P, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]),
    "scfft_region_mean_abs_b": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double)]),
    "scfft_probe_b": (C.c_int, [_P, _P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double)]),
    "scfft_get_state": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    "scfft_set_state": (C.c_int, [_P, _P, C.c_size_t]),
    "scfft_profile": (C.c_int, [_P, C.c_int32]),
    "scfft_profile_read": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "scfft_status_string": (C.c_char_p, [C.c_int]),
    "scfft_last_error": (C.c_char_p, [_P]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libscfft.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libscfft.so not built at %s: run __graft_entry__.build() or "
                          "python -m paper_1803_01346_amd.build" % path)
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


def _ptr(x):
    """Device address of a torch tensor (or an int address)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(st, ctx=None):
    if st < 0:
        lib = load()
        msg = lib.scfft_last_error(ctx).decode() if ctx else ""
        raise ScfftError(st, (lib.scfft_status_string(st).decode() + ": " + msg).strip(": "))
    return st


# ---- structure builders ---------------------------------------------------

def make_grid(n, half_width_m):
    return Grid((C.c_int32 * 3)(*[int(v) for v in n]), (C.c_double * 3)(*[float(v) for v in half_width_m]))


def make_material(n_power, jc, e0=1e-4, rho_out=20.0, l_char_m=1.0):
    return Material(float(n_power), float(jc), float(e0), float(rho_out), float(l_char_m))


def make_drive(kind, direction=(0.0, 0.0, 1.0), amp_T=0.0, t_ramp_s=1.0, freq_hz=0.0,
               t_s=None, b_T=None):
    kinds = {"ramp_hold": DRIVE_RAMP_HOLD, "sine": DRIVE_SINE, "pwl": DRIVE_PWL}
    k = kinds[kind] if isinstance(kind, str) else int(kind)
    d = Drive()
    d.kind = k
    d.dir = (C.c_double * 3)(*[float(v) for v in direction])
    d.amp_T = float(amp_T)
    d.t_ramp_s = float(t_ramp_s)
    d.freq_hz = float(freq_hz)
    d.n_pts = 0
    if k == DRIVE_PWL:
        ts = np.ascontiguousarray(t_s, dtype=np.float64)
        bs = np.ascontiguousarray(b_T, dtype=np.float64).reshape(-1)
        d.n_pts = ts.size
        d._keep = (ts, bs)
        d.t_s = ts.ctypes.data_as(C.POINTER(C.c_double))
        d.b_T = bs.ctypes.data_as(C.POINTER(C.c_double))
    return d


def make_shapes(prims, l_char_m):
    """Shapes from primitive dicts in units of l (see workloads) -> metres."""
    kinds = {"box": SHAPE_BOX, "cylinder": SHAPE_CYLINDER, "sphere": SHAPE_SPHERE}
    arr = (Shape * max(1, len(prims)))()
    for i, p in enumerate(prims):
        arr[i].kind = kinds[p["kind"]]
        arr[i].op = OP_ADD if p["op"] == "add" else OP_SUB
        arr[i].axis = int(p.get("axis", 2))
        arr[i].center_m = (C.c_double * 3)(*[float(v) * l_char_m for v in p["center"]])
        arr[i].size_m = (C.c_double * 3)(*[float(v) * l_char_m for v in p["size"]])
    return arr, len(prims)


def default_rhs_opts(**kw):
    o = RhsOpts()
    load().scfft_default_rhs_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def default_ode_opts(**kw):
    o = OdeOpts()
    load().scfft_default_ode_opts(C.byref(o))
    bps = kw.pop("breakpoints_s", None)
    for k, v in kw.items():
        setattr(o, k, v)
    if bps is not None:
        arr = np.ascontiguousarray(bps, dtype=np.float64)
        o._keep = arr
        o.n_bp = arr.size
        o.breakpoints_s = arr.ctypes.data_as(C.POINTER(C.c_double))
    return o


# ---- thin wrappers with the C names ---------------------------------------

def scfft_units(material):
    t0, hs = C.c_double(), C.c_double()
    _check(load().scfft_units(C.byref(material), C.byref(t0), C.byref(hs)))
    return t0.value, hs.value


def scfft_drive_eval(drive, material, t_s):
    he, hd = (C.c_double * 3)(), (C.c_double * 3)()
    _check(load().scfft_drive_eval(C.byref(drive), C.byref(material), float(t_s), he, hd))
    return np.array(he[:]), np.array(hd[:])


def scfft_voxelize_host(grid, material, shapes, n_shapes):
    n = tuple(grid.n)
    mask = np.zeros((n[2], n[1], n[0]), dtype=np.uint8)
    _check(load().scfft_voxelize_host(C.byref(grid), C.byref(material), shapes, int(n_shapes),
                                      mask.ctypes.data_as(C.POINTER(C.c_uint8))))
    return mask


def scfft_bs23_host(y, t0, t1, f, opts):
    """Integrate y' = f(t, y) on the host with the library's controller."""
    y = np.ascontiguousarray(y, dtype=np.float64).copy()
    n = y.size

    def cb(_user, t, yp, out):
        yy = np.ctypeslib.as_array(yp, shape=(n,))
        oo = np.ctypeslib.as_array(out, shape=(n,))
        oo[:] = f(t, yy.copy())
        return 0

    st = OdeStats()
    cbf = HOST_RHS(cb)
    rc = load().scfft_bs23_host(n, y.ctypes.data_as(C.POINTER(C.c_double)), float(t0), float(t1),
                                cbf, None, C.byref(opts), C.byref(st))
    return rc, y, st


def scfft_create(grid, material, precision=F64, stream=None):
    ctx = C.c_void_p()
    _check(load().scfft_create(C.byref(ctx), C.byref(grid), C.byref(material), int(precision),
                               stream))
    return ctx


def scfft_destroy(ctx):
    load().scfft_destroy(ctx)


def scfft_workspace_size(ctx):
    b = C.c_size_t()
    _check(load().scfft_workspace_size(ctx, C.byref(b)), ctx)
    return b.value


def scfft_set_workspace(ctx, ws, nbytes):
    return _check(load().scfft_set_workspace(ctx, _ptr(ws), int(nbytes)), ctx)


def scfft_mask_betti_host(mask):
    """(b0, b1, b2) of a host mask [Nz][Ny][Nx] (nonzero = Omega)."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.ndim != 3:
        raise ValueError("mask must be 3-D [Nz][Ny][Nx]")
    n = (C.c_int32 * 3)(m.shape[2], m.shape[1], m.shape[0])
    b = (C.c_int64 * 3)()
    _check(load().scfft_mask_betti_host(n, m.ctypes.data_as(C.POINTER(C.c_uint8)), b))
    return tuple(int(v) for v in b)


def scfft_mask_betti(ctx):
    b = (C.c_int64 * 3)()
    _check(load().scfft_mask_betti(ctx, b), ctx)
    return tuple(int(v) for v in b)


def scfft_voxelize(ctx, shapes, n_shapes):
    return _check(load().scfft_voxelize(ctx, shapes, int(n_shapes)), ctx)


def scfft_set_mask(ctx, dev_mask):
    return _check(load().scfft_set_mask(ctx, _ptr(dev_mask)), ctx)


def scfft_set_jc_map(ctx, dev_kappa):
    return _check(load().scfft_set_jc_map(ctx, _ptr(dev_kappa)), ctx)


def scfft_set_drive(ctx, drive):
    return _check(load().scfft_set_drive(ctx, C.byref(drive)), ctx)


def scfft_set_field_law(ctx, b0_T, alpha=1.0):
    return _check(load().scfft_set_field_law(ctx, float(b0_T), float(alpha)), ctx)


def scfft_set_anisotropy(ctx, weights=None):
    """Anisotropic law weights (a_x, a_y, a_z); None restores the isotropic law."""
    if weights is None:
        return _check(load().scfft_set_anisotropy(ctx, None), ctx)
    w = (C.c_double * 3)(*[float(v) for v in weights])
    return _check(load().scfft_set_anisotropy(ctx, w), ctx)


def scfft_set_rhs_opts(ctx, opts):
    return _check(load().scfft_set_rhs_opts(ctx, C.byref(opts)), ctx)


def scfft_reset_warm(ctx):
    return _check(load().scfft_reset_warm(ctx), ctx)


def scfft_init_state(ctx, t0_s, h):
    return _check(load().scfft_init_state(ctx, float(t0_s), _ptr(h)), ctx)


def scfft_rhs_eval(ctx, t_s, h, hdot, stats=None):
    return _check(load().scfft_rhs_eval(ctx, float(t_s), _ptr(h), _ptr(hdot),
                                        C.byref(stats) if stats is not None else None), ctx)


def scfft_integrate(ctx, t0_s, t1_s, h, opts, observer=None, stats=None):
    obs = OBSERVER(observer) if observer is not None else OBSERVER()
    return _check(load().scfft_integrate(ctx, float(t0_s), float(t1_s), _ptr(h), C.byref(opts),
                                         obs, None, C.byref(stats) if stats is not None else None),
                  ctx)


def scfft_curl(ctx, v, out):
    return _check(load().scfft_curl(ctx, _ptr(v), _ptr(out)), ctx)


def scfft_curl_noalloc(ctx, v, out):
    return _check(load().scfft_curl_noalloc(ctx, _ptr(v), _ptr(out)), ctx)


def scfft_phi(ctx, v, out):
    return _check(load().scfft_phi(ctx, _ptr(v), _ptr(out)), ctx)


def scfft_current(ctx, h, j):
    return _check(load().scfft_current(ctx, _ptr(h), _ptr(j)), ctx)


def scfft_moment(ctx, h, omega_only=0):
    m = (C.c_double * 3)()
    _check(load().scfft_moment(ctx, _ptr(h), int(omega_only), m), ctx)
    return np.array(m[:])


def scfft_step_moment(ctx, omega_only=0):
    m = (C.c_double * 3)()
    _check(load().scfft_step_moment(ctx, int(omega_only), m), ctx)
    return np.array(m[:])


def scfft_get_rhs_opts(ctx):
    o = RhsOpts()
    _check(load().scfft_get_rhs_opts(ctx, C.byref(o)), ctx)
    return o


def scfft_autotune(ctx, h, calls=5):
    """Returns (fuse_xy chosen, ms per call)."""
    fx = C.c_int32()
    ms = C.c_double()
    _check(load().scfft_autotune(ctx, _ptr(h), int(calls), C.byref(fx), C.byref(ms)), ctx)
    return fx.value, ms.value


def scfft_graph_moments(ctx, max_steps, omega_only=0):
    """Moments (A m^2) of the states accepted by the last waited graph
    integration: array [accepted][3]."""
    m = np.zeros((max(1, int(max_steps)), 3))
    n = C.c_int32()
    _check(load().scfft_graph_moments(ctx, int(omega_only), int(max_steps),
                                      m.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)), ctx)
    return m[:min(int(max_steps), n.value)]


def scfft_graph_workspace_size(ctx, steps):
    n = C.c_size_t()
    _check(load().scfft_graph_workspace_size(ctx, int(steps), C.byref(n)), ctx)
    return n.value


def scfft_integrate_graph(ctx, t0_s, t1_s, steps, graph_ws, h):
    nbytes = graph_ws.numel() * graph_ws.element_size()
    return _check(load().scfft_integrate_graph(ctx, float(t0_s), float(t1_s), int(steps), _ptr(graph_ws),
                                               nbytes, _ptr(h)), ctx)


def scfft_integrate_wait(ctx, stats=None):
    return _check(load().scfft_integrate_wait(ctx, C.byref(stats) if stats is not None else None), ctx)


def _bcheck(st, batch):
    if st < 0:
        msg = load().scfft_batch_last_error(batch).decode()
        raise ScfftError(st, "%s: %s" % (scfft_status_string(st), msg))
    return st


def scfft_batch_create(ctxs):
    arr = (_P * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    b = _P()
    st = load().scfft_batch_create(C.byref(b), arr, len(ctxs))
    if st < 0:
        raise ScfftError(st, "%s: %s" % (scfft_status_string(st), scfft_last_error(ctxs[0])))
    return b


def scfft_batch_destroy(batch):
    load().scfft_batch_destroy(batch)


def scfft_batch_rhs_eval(batch, t_s, h, hdot, field_stride):
    return _bcheck(load().scfft_batch_rhs_eval(batch, float(t_s), _ptr(h), _ptr(hdot), int(field_stride)), batch)


def scfft_batch_graph_workspace_size(batch, steps):
    n = C.c_size_t()
    _bcheck(load().scfft_batch_graph_workspace_size(batch, int(steps), C.byref(n)), batch)
    return n.value


def scfft_batch_integrate_graph(batch, t0_s, t1_s, steps, ws, h, field_stride):
    return _bcheck(load().scfft_batch_integrate_graph(batch, float(t0_s), float(t1_s), int(steps), _ptr(ws),
                                                      int(ws.numel()), _ptr(h), int(field_stride)), batch)


def scfft_batch_integrate_wait(batch, count):
    stats = (OdeStats * count)()
    _bcheck(load().scfft_batch_integrate_wait(batch, stats), batch)
    return list(stats)


def device_buffer(nbytes):
    """A 256-byte aligned uint8 device tensor of nbytes (workspaces)."""
    import torch
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


def scfft_rhs_vjp(ctx, h, warm_used, lam, mu, hbar, wbar=None, kappa_bar=None):
    """Returns (n_bar, hedot_bar); hbar (and wbar) are written, kappa_bar is
    accumulated."""
    nb = C.c_double()
    hb = (C.c_double * 3)()
    _check(load().scfft_rhs_vjp(ctx, _ptr(h), int(warm_used), _ptr(lam), _ptr(mu), _ptr(hbar),
                                _ptr(wbar), _ptr(kappa_bar), C.byref(nb), hb), ctx)
    return nb.value, np.array(hb[:])


def scfft_adjoint_workspace_size(ctx, steps, checkpoint_every):
    n = C.c_size_t()
    _check(load().scfft_adjoint_workspace_size(ctx, int(steps), int(checkpoint_every), C.byref(n)), ctx)
    return n.value


def scfft_integrate_adjoint(ctx, t0_s, t1_s, steps, checkpoint_every, adj_ws, h0, hT_bar, hT,
                            h0_bar, kappa_bar=None, want_p_bar=True):
    """Returns (n_bar, p_bar or None); hT, h0_bar written, kappa_bar accumulated."""
    nb = C.c_double()
    pb = (C.c_double * 3)()
    nbytes = adj_ws.numel() * adj_ws.element_size()
    _check(load().scfft_integrate_adjoint(ctx, float(t0_s), float(t1_s), int(steps),
                                          int(checkpoint_every), _ptr(adj_ws), nbytes, _ptr(h0),
                                          _ptr(hT_bar), _ptr(hT), _ptr(h0_bar), _ptr(kappa_bar),
                                          C.byref(nb), pb if want_p_bar else None), ctx)
    return nb.value, (np.array(pb[:]) if want_p_bar else None)


def scfft_region_mean_abs_b(ctx, h, dev_region):
    b = C.c_double()
    _check(load().scfft_region_mean_abs_b(ctx, _ptr(h), _ptr(dev_region), C.byref(b)), ctx)
    return b.value


def scfft_stray_fraction(ctx, h):
    f = C.c_double()
    _check(load().scfft_stray_fraction(ctx, _ptr(h), C.byref(f)), ctx)
    return f.value


def scfft_probe_b(ctx, h, xyz_m):
    pts = np.ascontiguousarray(xyz_m, dtype=np.float64).reshape(-1, 3)
    out = np.zeros_like(pts)
    _check(load().scfft_probe_b(ctx, _ptr(h), pts.ctypes.data_as(C.POINTER(C.c_double)),
                                pts.shape[0], out.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return out


def scfft_get_state(ctx):
    n = C.c_size_t()
    _check(load().scfft_get_state(ctx, None, C.byref(n)), ctx)
    buf = (C.c_char * n.value)()
    _check(load().scfft_get_state(ctx, buf, C.byref(n)), ctx)
    return bytes(buf)


def scfft_set_state(ctx, blob):
    buf = C.create_string_buffer(blob, len(blob))
    return _check(load().scfft_set_state(ctx, buf, len(blob)), ctx)


KERNEL_KINDS = ["X_FWD", "X_LAW", "X_HIN", "X_MASK", "X_UPDATE", "X_UPDATE_LAST", "X_STORE",
                "X_MOMENT", "Y_FWD", "Y_INV", "Z_CURL", "Z_PHI", "XY_FWD", "XY_HIN", "XY_MASK",
                "XY_UPDATE", "XY_UPDATE_LAST", "XY_STORE", "X_ADJ_START", "X_ADJ_ACC", "X_ADJ_LAST",
                "X_ADJ_LAW"]


def scfft_profile(ctx, enable):
    return _check(load().scfft_profile(ctx, int(enable)), ctx)


def scfft_profile_read(ctx):
    """{kind name: (launches, total_ms, total_algorithmic_bytes)}"""
    n = len(KERNEL_KINDS)
    la, ms, by = (C.c_int64 * n)(), (C.c_double * n)(), (C.c_double * n)()
    _check(load().scfft_profile_read(ctx, la, ms, by), ctx)
    return {k: (la[i], ms[i], by[i]) for i, k in enumerate(KERNEL_KINDS)}


def scfft_status_string(st):
    return load().scfft_status_string(int(st)).decode()


def scfft_last_error(ctx):
    return load().scfft_last_error(ctx).decode()


# ---- convenience ----------------------------------------------------------

class Simulation:
    """A context with its workspace tensor on the current torch device/stream.

    cfg: a dict with n, l_m, half_width (units of l), shapes (units of l),
    n_power, jc, e0, rho_out and drive (see workloads.CONFIGS).
    """

    def __init__(self, cfg, precision=F64, stream=None, rhs_opts=None, workspace=None):
        """workspace: (device address, bytes) of caller memory to use instead
        of a tensor of its own (the slices of a Batch)."""
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        self.dtype = torch.float64 if precision == F64 else torch.float32
        l = cfg["l_m"]
        self.grid = make_grid(cfg["n"], [v * l for v in cfg["half_width"]])
        self.material = make_material(cfg["n_power"], cfg["jc"], cfg.get("e0", 1e-4),
                                      cfg["rho_out"], l)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.ctx = scfft_create(self.grid, self.material, precision, stream)
        nbytes = scfft_workspace_size(self.ctx)
        if workspace is None:
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
        else:
            self.workspace = None
            aligned, have = workspace
            if have < nbytes:
                raise ValueError("workspace slice of %d bytes, %d needed" % (have, nbytes))
        scfft_set_workspace(self.ctx, aligned, nbytes)
        self.shapes, self.n_shapes = make_shapes(cfg["shapes"], l)
        if scfft_voxelize(self.ctx, self.shapes, self.n_shapes) == WARN_TOPOLOGY:
            warnings.warn("Omega is not contourwise simply connected (Betti numbers %s): "
                          "the method assumes it is" % (scfft_mask_betti(self.ctx),), stacklevel=2)
        d = dict(cfg["drive"])
        self.drive = make_drive(d.pop("kind"), **d)
        scfft_set_drive(self.ctx, self.drive)
        if rhs_opts is not None:
            scfft_set_rhs_opts(self.ctx, rhs_opts)
        self.t0_s, self.h_scale = scfft_units(self.material)

    @property
    def field_shape(self):
        n = self.cfg["n"]
        return (3, n[2], n[1], n[0])

    def empty_field(self):
        return self.torch.empty(self.field_shape, dtype=self.dtype, device="cuda")

    def mask_host(self):
        return scfft_voxelize_host(self.grid, self.material, self.shapes, self.n_shapes)

    def rhs_eval(self, t_s, h, hdot=None, stats=None):
        if hdot is None:
            hdot = self.empty_field()
        self._check_field(h)
        self._check_field(hdot)
        st = scfft_rhs_eval(self.ctx, t_s, h, hdot, stats)
        return hdot, st

    def _check_field(self, f):
        if tuple(f.shape) != self.field_shape or f.dtype != self.dtype or not f.is_contiguous():
            raise ValueError("field must be a contiguous %s tensor of shape %s"
                             % (self.dtype, self.field_shape))

    def close(self):
        if self.ctx:
            scfft_destroy(self.ctx)
            self.ctx = None


class Batch:
    """Same-size instances advanced with batched launches (scfft_batch_*):
    one Simulation per configuration, their workspaces carved in equal
    slices from one allocation.  Fields are tensors of shape
    (count, 3, Nz, Ny, Nx)."""

    def __init__(self, cfgs, precision=F64, stream=None, rhs_opts=None):
        import torch
        self.torch = torch
        l0 = cfgs[0]["l_m"]
        g = make_grid(cfgs[0]["n"], [v * l0 for v in cfgs[0]["half_width"]])
        m = make_material(cfgs[0]["n_power"], cfgs[0]["jc"], cfgs[0].get("e0", 1e-4), cfgs[0]["rho_out"], l0)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        ctx = scfft_create(g, m, precision, stream)
        stride = (scfft_workspace_size(ctx) + 255) // 256 * 256
        scfft_destroy(ctx)
        self.count = len(cfgs)
        self.stride = stride
        self.workspace = torch.empty(self.count * stride + 256, dtype=torch.uint8, device="cuda")
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        self.sims = [Simulation(c, precision=precision, stream=stream, rhs_opts=rhs_opts,
                                workspace=(base + b * stride, stride)) for b, c in enumerate(cfgs)]
        self.dtype = self.sims[0].dtype
        self.field_shape = (self.count,) + self.sims[0].field_shape
        self.field_stride = int(np.prod(self.sims[0].field_shape))
        self.batch = scfft_batch_create([s.ctx for s in self.sims])

    def empty_field(self):
        return self.torch.empty(self.field_shape, dtype=self.dtype, device="cuda")

    def _check_field(self, f):
        if tuple(f.shape) != self.field_shape or f.dtype != self.dtype or not f.is_contiguous():
            raise ValueError("field must be a contiguous %s tensor of shape %s" % (self.dtype, self.field_shape))

    def rhs_eval(self, t_s, h, hdot=None):
        if hdot is None:
            hdot = self.empty_field()
        self._check_field(h)
        self._check_field(hdot)
        scfft_batch_rhs_eval(self.batch, t_s, h, hdot, self.field_stride)
        return hdot

    def graph_workspace(self, steps):
        return device_buffer(scfft_batch_graph_workspace_size(self.batch, steps))

    def integrate_graph(self, t0_s, t1_s, steps, h, ws=None):
        """Enqueue `steps` fixed Bogacki-Shampine steps of every member; wait()
        returns the per-member stats and leaves the states in h."""
        self._check_field(h)
        self._ws = ws if ws is not None else self.graph_workspace(steps)
        scfft_batch_integrate_graph(self.batch, t0_s, t1_s, steps, self._ws, h, self.field_stride)

    def wait(self):
        return scfft_batch_integrate_wait(self.batch, self.count)

    def close(self):
        if self.batch:
            scfft_batch_destroy(self.batch)
            self.batch = None
        for s in self.sims:
            s.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
