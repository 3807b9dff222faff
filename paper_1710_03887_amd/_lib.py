"""ctypes binding of libdg.so with the same names as the C ABI (include/dg.h).

Only argument marshalling happens here: numpy arrays become host pointers,
torch tensors become device pointers, torch streams become hipStream_t.
Every step of the method runs in the library's HIP kernels; there is no
fallback: if the library is missing, importing this module raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DG_LIBRARY", os.path.join(HERE, "libdg.so"))

DG_OK, DG_EINVAL, DG_EMESH, DG_ENOMEM, DG_EHIP, DG_ENONPHYS, DG_ENODEV = 0, -1, -2, -3, -4, -5, -6
DG_BC_INTERIOR, DG_BC_OUTFLOW_CHAR, DG_BC_PASSTHRU, DG_BC_WALL, DG_BC_INFLOW, DG_BC_LEARNED = range(6)
DG_FP32, DG_SPLIT_BF16 = 0, 1
DG_SETUP_HOST_ONLY = 1
DG_SETUP_QUADRATURE = 2
DG_MLP_NOALLOC_ROWS = 4096

_ERRNAMES = {DG_EINVAL: "DG_EINVAL", DG_EMESH: "DG_EMESH", DG_ENOMEM: "DG_ENOMEM",
             DG_EHIP: "DG_EHIP", DG_ENONPHYS: "DG_ENONPHYS", DG_ENODEV: "DG_ENODEV"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python paper_1710_03887_amd/build.py`")
# torch carries its own HIP runtime under the same soname (libamdhip64.so.7);
# loading torch first makes libdg.so bind to that one, so that the library
# and torch's tensors and streams share a single runtime in the process.
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class dg_mesh_desc(ctypes.Structure):
    _fields_ = [("N", _i32), ("precision", _i32), ("K", _i64),
                ("xyz", _vp), ("EToV", _vp), ("bc", _vp),
                ("gamma", _f64), ("rho0", _f64), ("u0", _f64 * 3), ("p0", _f64),
                ("inflow_amp", _f64), ("inflow_alpha", _f64),
                ("flags", _i32), ("reserved", _i32)]


_SIGS = {
    "dg_mesh_setup": (ctypes.c_int, [ctypes.POINTER(dg_mesh_desc), _vp, ctypes.POINTER(_vp)]),
    "dg_destroy": (ctypes.c_int, [_vp]),
    "dg_last_error": (ctypes.c_char_p, [_vp]),
    "dg_sizes": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64)]),
    "dg_nodes": (ctypes.c_int, [_vp, _vp]),
    "dg_reference_operators": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "dg_geometry": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "dg_rhs": (ctypes.c_int, [_vp, _vp, _vp, _f64, _vp]),
    "dg_step": (ctypes.c_int, [_vp, _vp, _vp, _f64, _f64, _vp]),
    "dg_run": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f64, ctypes.POINTER(_f64),
                              ctypes.POINTER(_f64), _vp]),
    "dg_stage": (ctypes.c_int, [_vp, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _vp]),
    "dg_last_step": (_i64, [_vp]),
    "dg_stable_dt": (ctypes.c_int, [_vp, _vp, _f64, ctypes.POINTER(_f64), _vp]),
    "dg_prim_to_state": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "dg_state_to_prim": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "dg_set_launch": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _vp,
                                       ctypes.POINTER(_vp)]),
    "dg_batch_destroy": (ctypes.c_int, [_vp]),
    "dg_batch_last_error": (ctypes.c_char_p, [_vp]),
    "dg_batch_run": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _i64, _f64,
                                    _vp, _vp]),
    "dg_batch_first_bad": (ctypes.c_int, [_vp, _vp]),
    "dg_batch_set_launch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "dg_autotune": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int), _vp]),
    "dg_batch_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                         ctypes.c_char_p, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int), _vp]),
    "dg_set_kernel": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dg_get_kernel": (ctypes.c_int, [_vp]),
    "dg_run_fixed": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f64, ctypes.POINTER(_f64), _vp]),
    "dg_mlp_create": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    "dg_mlp_destroy": (ctypes.c_int, [_vp]),
    "dg_mlp_last_error": (ctypes.c_char_p, [_vp]),
    "dg_mlp_get_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_mlp_set_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "dg_mlp_infer": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_int, _vp]),
    "dg_mlp_infer_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp]),
    "dg_mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(ctypes.c_float), _vp, _vp]),
    "dg_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_float), _vp]),
    "dg_set_learned_bc": (ctypes.c_int, [_vp, _vp, _f64, _f64, _f64, _f64]),
    "dg_learned_faces": (_i64, [_vp, _vp]),
    "dg_sample_traces": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f64, _vp, _vp, _vp]),
    "dg_set_damping": (ctypes.c_int, [_vp, _vp]),
    "dg_set_curved": (ctypes.c_int, [_vp, _vp, _f64, ctypes.POINTER(_i64), _vp]),
    "dg_probe_setup": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "dg_probe_sample": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "dg_run_probes": (ctypes.c_int, [_vp, _vp, _vp, _i64, _f64, ctypes.POINTER(_f64), _vp, _vp]),
    "dg_spectrum": (ctypes.c_int, [_vp, _i64, _i32, _f64, _vp, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code, handle):
    if code != DG_OK:
        msg = _lib.dg_last_error(handle)
        raise DGError(code, msg.decode() if msg else "")


def _ptr(x):
    """Device pointer of a torch tensor, or host pointer of a numpy array."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"cannot pass {type(x)}")


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # torch absent or no device: default stream
            pass
        return None
    return getattr(stream, "cuda_stream", stream)


def _check_state(ctx, x, name):
    if x is None:
        raise ValueError(f"{name} is None")
    shape = (ctx.K, 5, ctx.Np)
    if tuple(x.shape) != shape:
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {shape}")
    if str(getattr(x, "dtype", "")) not in ("torch.float32", "float32"):
        raise ValueError(f"{name} must be float32")
    if not getattr(x, "is_cuda", False):
        raise ValueError(f"{name} must be a device tensor")


class Context:
    """Owns a dg_ctx handle; freed by dg_destroy."""

    def __init__(self, handle, N):
        self.handle = handle
        self.N = N
        Np, Nfp, K = _i32(), _i32(), _i64()
        _check(_lib.dg_sizes(handle, ctypes.byref(Np), ctypes.byref(Nfp), ctypes.byref(K)), handle)
        self.Np, self.Nfp, self.K = Np.value, Nfp.value, K.value

    def close(self):
        if self.handle:
            _lib.dg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dg_mesh_setup(xyz, EToV, bc, N, gamma=1.4, rho0=1.0, u0=(0.0, 0.0, 0.0), p0=1.0 / 1.4,
                  precision=DG_FP32, inflow_amp=0.0, inflow_alpha=2 * np.pi * 565.0 / 343.0,
                  host_only=False, quadrature=False, stream=None):
    """Set up a mesh; quadrature=True selects the weak form with Gauss
    quadrature and RK2 (DG_SETUP_QUADRATURE) instead of the nodal scheme."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    EToV = np.ascontiguousarray(EToV, dtype=np.int64)
    bc = np.ascontiguousarray(bc, dtype=np.int8)
    K = xyz.shape[0]
    if xyz.shape != (K, 4, 3) or EToV.shape != (K, 4) or bc.shape != (K, 4):
        raise ValueError("mesh arrays must be xyz[K,4,3], EToV[K,4], bc[K,4]")
    d = dg_mesh_desc(N=N, precision=precision, K=K, xyz=xyz.ctypes.data, EToV=EToV.ctypes.data,
                     bc=bc.ctypes.data, gamma=gamma, rho0=rho0, u0=(_f64 * 3)(*u0), p0=p0,
                     inflow_amp=inflow_amp, inflow_alpha=inflow_alpha,
                     flags=(DG_SETUP_HOST_ONLY if host_only else 0) |
                     (DG_SETUP_QUADRATURE if quadrature else 0), reserved=0)
    h = _vp()
    _check(_lib.dg_mesh_setup(ctypes.byref(d), None if host_only else _stream(stream),
                              ctypes.byref(h)), None)
    return Context(h, N)


def dg_destroy(ctx):
    ctx.close()


def dg_last_error(ctx=None):
    msg = _lib.dg_last_error(ctx.handle if ctx else None)
    return msg.decode() if msg else ""


def dg_sizes(ctx):
    return ctx.Np, ctx.Nfp, ctx.K


def dg_nodes(ctx):
    out = np.empty((ctx.K, ctx.Np, 3))
    _check(_lib.dg_nodes(ctx.handle, _ptr(out)), ctx.handle)
    return out


def dg_reference_operators(ctx):
    Np, Nfp = ctx.Np, ctx.Nfp
    rst = np.empty((Np, 3))
    Dr, Ds, Dt = (np.empty((Np, Np)) for _ in range(3))
    LIFT = np.empty((Np, 4 * Nfp))
    Fmask = np.empty((4, Nfp), dtype=np.int32)
    _check(_lib.dg_reference_operators(ctx.handle, *(_ptr(a) for a in (rst, Dr, Ds, Dt, LIFT, Fmask))),
           ctx.handle)
    return {"rst": rst, "Dr": Dr, "Ds": Ds, "Dt": Dt, "LIFT": LIFT, "Fmask": Fmask}


def dg_geometry(ctx):
    K, Nfp = ctx.K, ctx.Nfp
    g = {"drst_dx": np.empty((K, 3, 3)), "J": np.empty(K), "nrm": np.empty((K, 4, 3)),
         "Fscale": np.empty((K, 4)), "mapP": np.empty((K, 4, Nfp), dtype=np.int64)}
    _check(_lib.dg_geometry(ctx.handle, *(_ptr(g[k]) for k in ("drst_dx", "J", "nrm", "Fscale", "mapP"))),
           ctx.handle)
    return g


def dg_rhs(ctx, q, rhs, t=0.0, stream=None):
    _check_state(ctx, q, "q")
    _check_state(ctx, rhs, "rhs")
    _check(_lib.dg_rhs(ctx.handle, _ptr(q), _ptr(rhs), float(t), _stream(stream)), ctx.handle)


def dg_step(ctx, q, res, t, dt, stream=None):
    _check_state(ctx, q, "q")
    _check_state(ctx, res, "res")
    _check(_lib.dg_step(ctx.handle, _ptr(q), _ptr(res), float(t), float(dt), _stream(stream)),
           ctx.handle)


def dg_stage(ctx, q_in, q_out, res, a, b, t_stage, dt, stream=None):
    for x, nm in ((q_in, "q_in"), (q_out, "q_out"), (res, "res")):
        _check_state(ctx, x, nm)
    _check(_lib.dg_stage(ctx.handle, _ptr(q_in), _ptr(q_out), _ptr(res), float(a), float(b),
                         float(t_stage), float(dt), _stream(stream)), ctx.handle)


def dg_run(ctx, q, res, nsteps, cfl, t=0.0, stream=None):
    """Returns (t_end, dt_last).  Raises DGError(DG_ENONPHYS) on a
    non-physical state; dg_last_step(ctx) then names the first such step."""
    _check_state(ctx, q, "q")
    _check_state(ctx, res, "res")
    tt, dl = _f64(t), _f64(0.0)
    _check(_lib.dg_run(ctx.handle, _ptr(q), _ptr(res), int(nsteps), float(cfl), ctypes.byref(tt),
                       ctypes.byref(dl), _stream(stream)), ctx.handle)
    return tt.value, dl.value


def dg_last_step(ctx):
    return int(_lib.dg_last_step(ctx.handle))


def dg_stable_dt(ctx, q, cfl, stream=None):
    _check_state(ctx, q, "q")
    dt = _f64()
    _check(_lib.dg_stable_dt(ctx.handle, _ptr(q), float(cfl), ctypes.byref(dt), _stream(stream)),
           ctx.handle)
    return dt.value


def dg_prim_to_state(ctx, prim, q, stream=None):
    _check_state(ctx, prim, "prim")
    _check_state(ctx, q, "q")
    _check(_lib.dg_prim_to_state(ctx.handle, _ptr(prim), _ptr(q), _stream(stream)), ctx.handle)


def dg_state_to_prim(ctx, q, prim, stream=None):
    _check_state(ctx, q, "q")
    _check_state(ctx, prim, "prim")
    _check(_lib.dg_state_to_prim(ctx.handle, _ptr(q), _ptr(prim), _stream(stream)), ctx.handle)


def dg_set_kernel(ctx, variant):
    _check(_lib.dg_set_kernel(ctx.handle, int(variant)), ctx.handle)


def dg_get_kernel(ctx):
    return int(_lib.dg_get_kernel(ctx.handle))


def dg_set_launch(ctx, blocks_per_cu):
    _check(_lib.dg_set_launch(ctx.handle, int(blocks_per_cu)), ctx.handle)


# ---- batched ensembles --------------------------------------------------------
MEMBERS = 16


class Batch:
    """Owns a dg_batch handle; keeps its contexts alive."""

    def __init__(self, handle, geoms, members):
        self.handle = handle
        self.geoms = list(geoms)
        self.members = members

    def close(self):
        if self.handle:
            _lib.dg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(code, b):
    if code != DG_OK:
        msg = _lib.dg_batch_last_error(b.handle if b is not None else None)
        raise DGError(code, msg.decode() if msg else "")


def dg_batch_create(geoms, members=MEMBERS, stream=None):
    arr = (_vp * len(geoms))(*[g.handle for g in geoms])
    h = _vp()
    code = _lib.dg_batch_create(arr, len(geoms), int(members), _stream(stream), ctypes.byref(h))
    if code != DG_OK:
        raise DGError(code, "dg_batch_create: contexts must be device contexts with the same N "
                            "and ambient state; 1 <= members <= 16")
    return Batch(h, geoms, members)


def dg_batch_destroy(b):
    b.close()


def dg_batch_last_error(b):
    msg = _lib.dg_batch_last_error(b.handle)
    return msg.decode() if msg else ""


def _check_batch_state(ctx, x, name):
    shape = (ctx.K, 5, ctx.Np, MEMBERS)
    if x is None or tuple(x.shape) != shape:
        raise ValueError(f"{name} must have shape {shape}")
    if str(x.dtype) != "torch.float32" or not x.is_cuda or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 device tensor")


def dg_batch_run(b, q, res, amps, nsteps, cfl, t=None, stream=None):
    """q, res: one [K_g, 5, Np, 16] float32 device tensor per geometry;
    amps: [ngeom, 16] inflow amplitudes; t: [ngeom, 16] start times (zeros
    when None).  Returns the end times [ngeom, 16].  Raises
    DGError(DG_ENONPHYS) when a member met a non-physical state
    (dg_batch_first_bad names the steps)."""
    ng = len(b.geoms)
    if len(q) != ng or len(res) != ng:
        raise ValueError("one state and one residual per geometry")
    for g, ctx in enumerate(b.geoms):
        _check_batch_state(ctx, q[g], f"q[{g}]")
        _check_batch_state(ctx, res[g], f"res[{g}]")
    amps = np.ascontiguousarray(np.broadcast_to(np.asarray(amps, dtype=np.float64), (ng, MEMBERS)))
    tt = np.zeros((ng, MEMBERS)) if t is None else np.array(np.broadcast_to(t, (ng, MEMBERS)),
                                                               dtype=np.float64)
    qp = (_vp * ng)(*[x.data_ptr() for x in q])
    rp = (_vp * ng)(*[x.data_ptr() for x in res])
    _bcheck(_lib.dg_batch_run(b.handle, qp, rp, amps.ctypes.data, int(nsteps), float(cfl),
                              tt.ctypes.data, _stream(stream)), b)
    return tt


def dg_batch_first_bad(b):
    out = np.full((len(b.geoms), MEMBERS), -1, dtype=np.int64)
    _bcheck(_lib.dg_batch_first_bad(b.handle, out.ctypes.data), b)
    return out


def dg_batch_set_launch(b, blocks_per_cu, waves_per_block):
    _bcheck(_lib.dg_batch_set_launch(b.handle, int(blocks_per_cu), int(waves_per_block)), b)


def dg_autotune(ctx, q, res, cache_path=None, stream=None):
    """Pick the stage kernel's resident blocks per CU by timing; returns it."""
    _check_state(ctx, q, "q")
    _check_state(ctx, res, "res")
    bpc = ctypes.c_int()
    _check(_lib.dg_autotune(ctx.handle, _ptr(q), _ptr(res),
                            cache_path.encode() if cache_path else None, ctypes.byref(bpc),
                            _stream(stream)), ctx.handle)
    return bpc.value


def dg_batch_autotune(b, q, res, cache_path=None, stream=None):
    """Pick the batched stage kernel's launch shape by timing; returns
    (blocks_per_cu, waves_per_block)."""
    ng = len(b.geoms)
    for g, ctx in enumerate(b.geoms):
        _check_batch_state(ctx, q[g], f"q[{g}]")
        _check_batch_state(ctx, res[g], f"res[{g}]")
    qp = (_vp * ng)(*[x.data_ptr() for x in q])
    rp = (_vp * ng)(*[x.data_ptr() for x in res])
    bpc, w = ctypes.c_int(), ctypes.c_int()
    _bcheck(_lib.dg_batch_autotune(b.handle, qp, rp, cache_path.encode() if cache_path else None,
                                   ctypes.byref(bpc), ctypes.byref(w), _stream(stream)), b)
    return bpc.value, w.value


def dg_run_fixed(ctx, q, res, nsteps, dt, t=0.0, stream=None):
    """dg_run with a fixed time step dt; returns the end time."""
    _check_state(ctx, q, "q")
    _check_state(ctx, res, "res")
    tt = _f64(t)
    _check(_lib.dg_run_fixed(ctx.handle, _ptr(q), _ptr(res), int(nsteps), float(dt),
                             ctypes.byref(tt), _stream(stream)), ctx.handle)
    return tt.value


# ---- absorbing layer --------------------------------------------------------------------
def dg_set_damping(ctx, sigma):
    """Damping rate per node (device float32 [K, Np]) or None to turn the
    layer off; the tensor must stay alive while the context uses it."""
    if sigma is not None:
        _check_device_f32(sigma, (ctx.K, ctx.Np), "sigma")
    _check(_lib.dg_set_damping(ctx.handle, _ptr(sigma)), ctx.handle)
    ctx.sigma = sigma   # keeps the tensor alive with the context


def dg_set_curved(ctx, xyz_nodes, tol=1e-9, stream=None):
    """Curved node positions (host float64 [K, Np, 3], library node order)
    or None to clear; returns the number of curved elements."""
    n = _i64(0)
    if xyz_nodes is None:
        _check(_lib.dg_set_curved(ctx.handle, None, float(tol), ctypes.byref(n), _stream(stream)),
               ctx.handle)
        return 0
    x = np.ascontiguousarray(xyz_nodes, dtype=np.float64)
    if x.shape != (ctx.K, ctx.Np, 3):
        raise ValueError(f"xyz_nodes must have shape {(ctx.K, ctx.Np, 3)}")
    _check(_lib.dg_set_curved(ctx.handle, _ptr(x), float(tol), ctypes.byref(n), _stream(stream)),
           ctx.handle)
    return int(n.value)


# ---- pressure probes and spectra -----------------------------------------------------
def _check_device_f32(x, shape, name):
    if x is None or tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}")
    if str(getattr(x, "dtype", "")) != "torch.float32" or not getattr(x, "is_cuda", False):
        raise ValueError(f"{name} must be a float32 device tensor")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def dg_probe_setup(ctx, xyz, weights=False):
    """Locate points (array [n, 3]) and keep them as the probe set; returns
    the element index of each point (numpy int64 [n]) and, with weights,
    also their interpolation weights (numpy float64 [n, Np])."""
    pts = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    elems = np.empty(len(pts), dtype=np.int64)
    w = np.empty((len(pts), ctx.Np), dtype=np.float64) if weights else None
    _check(_lib.dg_probe_setup(ctx.handle, _ptr(pts), int(len(pts)), _ptr(elems), _ptr(w)),
           ctx.handle)
    ctx.n_probes = len(pts)
    return (elems, w) if weights else elems


def dg_probe_sample(ctx, q, out, stream=None):
    """p - p0 at every probe of state q into out (device float32 [n])."""
    _check_state(ctx, q, "q")
    _check_device_f32(out, (getattr(ctx, "n_probes", 0),), "out")
    _check(_lib.dg_probe_sample(ctx.handle, _ptr(q), _ptr(out), _stream(stream)), ctx.handle)


def dg_run_probes(ctx, q, res, nsteps, dt, t=0.0, series=None, stream=None):
    """dg_run with a fixed dt that records p - p0 at every probe after every
    step into series (device float32 [nsteps, n]); returns the end time."""
    _check_state(ctx, q, "q")
    _check_state(ctx, res, "res")
    _check_device_f32(series, (int(nsteps), getattr(ctx, "n_probes", 0)), "series")
    tt = _f64(t)
    _check(_lib.dg_run_probes(ctx.handle, _ptr(q), _ptr(res), int(nsteps), float(dt),
                              ctypes.byref(tt), _ptr(series), _stream(stream)), ctx.handle)
    return tt.value


def dg_spectrum(series, p_ref, db, stream=None):
    """Amplitude spectra in dB of the columns of series (device float32
    [n_samples, n_signals]) into db (device float32 [n_signals, n_samples//2 + 1])."""
    if series is None or series.dim() != 2:
        raise ValueError("series must be a 2-D device tensor")
    n, ns = series.shape
    _check_device_f32(series, (n, ns), "series")
    _check_device_f32(db, (ns, n // 2 + 1), "db")
    _check(_lib.dg_spectrum(_ptr(series), int(n), int(ns), float(p_ref), _ptr(db),
                            _stream(stream)), None)


# ---- learned boundary closure ------------------------------------------------------
DG_MLP_PARAMS = 36299
MLP_IN, MLP_OUT = 78, 75


class Mlp:
    """Owns a dg_mlp handle."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            _lib.dg_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mcheck(code, m):
    if code != DG_OK:
        msg = _lib.dg_mlp_last_error(m.handle if m is not None else None)
        raise DGError(code, msg.decode() if msg else "")


def _check_dev(x, shape, dtype, name):
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(shape)}")
    if str(x.dtype) != dtype or not x.is_cuda or not x.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor")


def dg_mlp_create(params, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.shape != (DG_MLP_PARAMS,):
        raise ValueError(f"params must have {DG_MLP_PARAMS} values")
    h = _vp()
    code = _lib.dg_mlp_create(p.ctypes.data, _stream(stream), ctypes.byref(h))
    if code != DG_OK:
        raise DGError(code, "dg_mlp_create")
    return Mlp(h)


def dg_mlp_destroy(m):
    m.close()


def dg_mlp_last_error(m):
    msg = _lib.dg_mlp_last_error(m.handle)
    return msg.decode() if msg else ""


def dg_mlp_get_params(m, stream=None):
    out = np.empty(DG_MLP_PARAMS, dtype=np.float32)
    _mcheck(_lib.dg_mlp_get_params(m.handle, out.ctypes.data, _stream(stream)), m)
    return out


def dg_mlp_set_params(m, params, stream=None):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.shape != (DG_MLP_PARAMS,):
        raise ValueError(f"params must have {DG_MLP_PARAMS} values")
    _mcheck(_lib.dg_mlp_set_params(m.handle, p.ctypes.data, _stream(stream)), m)


def dg_mlp_infer(m, X, Y, bf16=True, stream=None):
    B = X.shape[0]
    _check_dev(X, (B, MLP_IN), "torch.float32", "X")
    _check_dev(Y, (B, MLP_OUT), "torch.float32", "Y")
    _mcheck(_lib.dg_mlp_infer(m.handle, _ptr(X), _ptr(Y), B, 1 if bf16 else 0, _stream(stream)), m)


def dg_mlp_infer_noalloc(m, X, Y, stream=None):
    B = X.shape[0]
    _check_dev(X, (B, MLP_IN), "torch.float32", "X")
    _check_dev(Y, (B, MLP_OUT), "torch.float32", "Y")
    _mcheck(_lib.dg_mlp_infer_noalloc(m.handle, _ptr(X), _ptr(Y), B, _stream(stream)), m)


def dg_mlp_grad(m, X, Y, grads=None, stream=None):
    """Returns (loss, grads) with grads a device FP32 tensor."""
    import torch
    B = X.shape[0]
    _check_dev(X, (B, MLP_IN), "torch.float32", "X")
    _check_dev(Y, (B, MLP_OUT), "torch.float32", "Y")
    if grads is None:
        grads = torch.empty(DG_MLP_PARAMS, dtype=torch.float32, device=X.device)
    _check_dev(grads, (DG_MLP_PARAMS,), "torch.float32", "grads")
    loss = ctypes.c_float()
    _mcheck(_lib.dg_mlp_grad(m.handle, _ptr(X), _ptr(Y), B, ctypes.byref(loss), _ptr(grads),
                             _stream(stream)), m)
    return loss.value, grads


def dg_mlp_train_step(m, X, Y, lr, rows=None, batch=None, want_loss=True, stream=None):
    """One Adam step on rows `rows` (device int64) of the data set (X, Y),
    or on its first `batch` rows.  Returns the minibatch loss (or None)."""
    n = X.shape[0]
    _check_dev(X, (n, MLP_IN), "torch.float32", "X")
    _check_dev(Y, (n, MLP_OUT), "torch.float32", "Y")
    if rows is not None:
        _check_dev(rows, (rows.shape[0],), "torch.int64", "rows")
        B = rows.shape[0]
    else:
        B = n if batch is None else int(batch)
    loss = ctypes.c_float()
    _mcheck(_lib.dg_mlp_train_step(m.handle, _ptr(X), _ptr(Y), n, _ptr(rows), B, float(lr),
                                   ctypes.byref(loss) if want_loss else None, _stream(stream)), m)
    return loss.value if want_loss else None


def dg_set_learned_bc(ctx, m, norm, p_lo, p_hi, blend=1.0):
    _check(_lib.dg_set_learned_bc(ctx.handle, m.handle if m is not None else None, float(norm),
                                  float(p_lo), float(p_hi), float(blend)), ctx.handle)
    ctx.mlp = m          # keep the network alive while attached


def dg_learned_faces(ctx):
    n = _lib.dg_learned_faces(ctx.handle, None)
    out = np.empty(max(n, 0), dtype=np.int64)
    if n > 0:
        _lib.dg_learned_faces(ctx.handle, out.ctypes.data)
    return out


def dg_sample_traces(ctx, q, faces, norm, X, Y=None, stream=None):
    _check_state(ctx, q, "q")
    nf = faces.shape[0]
    _check_dev(faces, (nf,), "torch.int64", "faces")
    nfp = ctx.Nfp
    _check_dev(X, (nf, 5 * nfp + 3), "torch.float32", "X")
    if Y is not None:
        _check_dev(Y, (nf, 5 * nfp), "torch.float32", "Y")
    _check(_lib.dg_sample_traces(ctx.handle, _ptr(q), _ptr(faces), nf, float(norm), _ptr(X),
                                 _ptr(Y), _stream(stream)), ctx.handle)
