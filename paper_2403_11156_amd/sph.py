"""Thin ctypes binding of libsph.so (include/sph.h), same names as the C ABI.

Argument marshalling only: every step of the time step runs in the HIP
library.  If libsph.so is missing this module raises at import; there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsph.so")

SPH_OK = 0
SPH_ERR_INVALID, SPH_ERR_OOM, SPH_ERR_DEVICE, SPH_ERR_CAPACITY, SPH_ERR_STATE, SPH_ERR_NUMERIC = -1, -2, -3, -4, -5, -6

FIELD_X, FIELD_V, FIELD_RHO, FIELD_ALPHA = 1 << 0, 1 << 1, 1 << 2, 1 << 3
FIELD_K, FIELD_KV, FIELD_KAPPA, FIELD_ACCEL = 1 << 4, 1 << 5, 1 << 6, 1 << 7
FIELD_NBR, FIELD_PSI, FIELD_BOUNDARY, FIELD_RIGID = 1 << 8, 1 << 9, 1 << 10, 1 << 11
FIELD_DVISC = 1 << 12


class sph_params(C.Structure):
    _fields_ = [
        ("r", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
        ("gravity", C.c_double * 3),
        ("domain_min", C.c_double * 3), ("domain_max", C.c_double * 3),
        ("eta_density", C.c_double), ("eta_divergence", C.c_double),
        ("max_iters", C.c_int32),
        ("dt_max", C.c_double), ("cfl_lambda", C.c_double),
        ("visc_model", C.c_int32), ("visc", C.c_double),
        ("cg_tol", C.c_double), ("cg_max_iters", C.c_int32),
        ("warm_start", C.c_int32), ("warm_factor", C.c_double),
        ("max_neighbors", C.c_int32), ("max_boundary_neighbors", C.c_int32),
        ("auto_rebuild", C.c_int32),
        ("solver", C.c_int32), ("wcsph_k", C.c_double), ("wcsph_gamma", C.c_double),
        ("cg_warm_factor", C.c_double),
        ("separate_div_check", C.c_int32),
        ("alpha_max_factor", C.c_double),
        ("eta_density_max", C.c_double),
        ("rigid_coupling", C.c_int32),
        ("rigid_contact", C.c_int32),
    ]


class sph_rigid_desc(C.Structure):
    _fields_ = [("mass", C.c_double), ("inertia", C.c_double * 3), ("com", C.c_double * 3),
                ("quat", C.c_double * 4), ("vel", C.c_double * 3), ("omega", C.c_double * 3)]


class sph_scene(C.Structure):
    _fields_ = [
        ("n_fluid", C.c_int64), ("n_boundary", C.c_int64), ("n_rigid", C.c_int32),
        ("x_fluid", C.c_void_p), ("v_fluid", C.c_void_p), ("x_boundary", C.c_void_p),
        ("body_of_boundary", C.c_void_p), ("rigid", C.c_void_p),
        ("device_arena", C.c_void_p), ("device_arena_bytes", C.c_int64),
    ]


class sph_step_stats(C.Structure):
    _fields_ = [
        ("dt", C.c_double),
        ("iters_div", C.c_int32), ("iters_dens", C.c_int32),
        ("converged_div", C.c_int32), ("converged_dens", C.c_int32),
        ("err_div", C.c_double), ("err_dens", C.c_double),
        ("cg_iters", C.c_int32), ("cg_resid", C.c_double),
        ("nbr_min", C.c_int32), ("nbr_max", C.c_int32), ("nbr_mean", C.c_double),
        ("warm_fallback", C.c_int32), ("step_index", C.c_int64),
        ("err_dens_max", C.c_double),
    ]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class sph_host_view(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("v", C.c_void_p),
        ("rho", C.c_void_p), ("alpha", C.c_void_p), ("K", C.c_void_p), ("Kv", C.c_void_p),
        ("kappa", C.c_void_p), ("accel", C.c_void_p),
        ("n_fluid_nbrs", C.c_void_p), ("n_boundary_nbrs", C.c_void_p),
        ("psi", C.c_void_p), ("x_boundary", C.c_void_p), ("v_boundary", C.c_void_p),
        ("rigid", C.c_void_p), ("rigid_force", C.c_void_p), ("rigid_torque", C.c_void_p),
        ("dvisc", C.c_void_p),
    ]


class sph_info(C.Structure):
    _fields_ = [
        ("n_fluid", C.c_int64), ("n_boundary", C.c_int64), ("n_rigid", C.c_int32),
        ("grid_n", C.c_int32 * 3), ("cell", C.c_float), ("inv_cell", C.c_float),
        ("origin", C.c_float * 3), ("h2", C.c_float),
        ("max_neighbors", C.c_int32), ("max_boundary_neighbors", C.c_int32),
        ("device_bytes", C.c_int64),
    ]


class sph_nbr_view(C.Structure):
    _fields_ = [
        ("keys_f", C.c_void_p), ("perm_f", C.c_void_p), ("start_f", C.c_void_p),
        ("counts_f", C.c_void_p), ("lists_f", C.c_void_p),
        ("keys_b", C.c_void_p), ("perm_b", C.c_void_p), ("start_b", C.c_void_p),
        ("counts_b", C.c_void_p), ("lists_b", C.c_void_p),
        ("cap_f", C.c_int64), ("cap_b", C.c_int64),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the HIP library is required, there is no fallback)")
    # torch first: it ships its own HIP runtime, and the library must bind to
    # that same runtime (loaded first, the library would pull in the system's
    # copy, and torch's streams and memory would then be foreign to it)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "sph_create": (C.c_int, [C.POINTER(sph_params), C.POINTER(sph_scene), P, C.POINTER(P)]),
        "sph_required_bytes": (C.c_int, [C.POINTER(sph_params), C.POINTER(sph_scene), C.POINTER(C.c_int64)]),
        "sph_destroy": (None, [P]),
        "sph_build_neighbors": (C.c_int, [P]),
        "sph_step": (C.c_int, [P, C.POINTER(sph_step_stats)]),
        "sph_read_state": (C.c_int, [P, C.c_uint32, C.POINTER(sph_host_view)]),
        "sph_write_state": (C.c_int, [P, C.c_uint32, C.POINTER(sph_host_view)]),
        "sph_get_info": (C.c_int, [P, C.POINTER(sph_info)]),
        "sph_read_neighbors": (C.c_int, [P, C.POINTER(sph_nbr_view)]),
        "sph_set_forced_iters": (C.c_int, [P, C.c_int32, C.c_int32]),
        "sph_profile_enable": (C.c_int, [P, C.c_int32]),
        "sph_profile_only": (C.c_int, [P, C.c_char_p]),
        "sph_profile_read": (C.c_int, [P, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]),
        "sph_last_error": (C.c_char_p, [P]),
        "sph_mlp_create": (C.c_int, [P, P, C.POINTER(P)]),
        "sph_mlp_destroy": (None, [P]),
        "sph_mlp_get_params": (C.c_int, [P, P]),
        "sph_mlp_set_params": (C.c_int, [P, P]),
        "sph_mlp_forward": (C.c_int, [P, P, P, C.c_int64]),
        "sph_mlp_grad": (C.c_int, [P, P, P, C.c_int64, P, C.POINTER(C.c_double)]),
        "sph_mlp_train_step": (C.c_int, [P, P, P, C.c_int64, C.c_float, C.POINTER(C.c_double)]),
        "sph_mlp_grad_noalloc": (C.c_int, [P, P, P, C.c_int64, P, P, P]),
        "sph_set_warm_start": (C.c_int, [P, C.c_int32, P]),
        "sph_enable_trace": (C.c_int, [P, P, P, C.c_int64]),
        "sph_trace_rows": (C.c_int, [P, C.POINTER(C.c_int64)]),
        "sph_strerror": (C.c_char_p, [C.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()

# the C entry points under their own names
sph_create = lib.sph_create
sph_required_bytes = lib.sph_required_bytes
sph_destroy = lib.sph_destroy
sph_build_neighbors = lib.sph_build_neighbors
sph_step = lib.sph_step
sph_read_state = lib.sph_read_state
sph_write_state = lib.sph_write_state
sph_get_info = lib.sph_get_info
sph_read_neighbors = lib.sph_read_neighbors
sph_set_forced_iters = lib.sph_set_forced_iters
sph_profile_enable = lib.sph_profile_enable
sph_profile_only = lib.sph_profile_only
sph_profile_read = lib.sph_profile_read
sph_last_error = lib.sph_last_error
sph_strerror = lib.sph_strerror
sph_mlp_create = lib.sph_mlp_create
sph_mlp_destroy = lib.sph_mlp_destroy
sph_mlp_get_params = lib.sph_mlp_get_params
sph_mlp_set_params = lib.sph_mlp_set_params
sph_mlp_forward = lib.sph_mlp_forward
sph_mlp_grad = lib.sph_mlp_grad
sph_mlp_train_step = lib.sph_mlp_train_step
sph_mlp_grad_noalloc = lib.sph_mlp_grad_noalloc
sph_set_warm_start = lib.sph_set_warm_start
sph_enable_trace = lib.sph_enable_trace
sph_trace_rows = lib.sph_trace_rows

MLP_PARAMS = 4620


class SphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{sph_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(pd: Dict) -> sph_params:
    p = sph_params()
    p.r, p.h, p.rho0 = pd["r"], pd["h"], pd["rho0"]
    for a in range(3):
        p.gravity[a] = pd["gravity"][a]
        p.domain_min[a] = pd["domain_min"][a]
        p.domain_max[a] = pd["domain_max"][a]
    p.eta_density, p.eta_divergence = pd["eta_density"], pd["eta_divergence"]
    p.max_iters = pd["max_iters"]
    p.dt_max, p.cfl_lambda = pd["dt_max"], pd["cfl_lambda"]
    p.visc_model, p.visc = pd["visc_model"], pd["visc"]
    p.cg_tol, p.cg_max_iters = pd["cg_tol"], pd["cg_max_iters"]
    p.warm_start, p.warm_factor = pd["warm_start"], pd["warm_factor"]
    p.max_neighbors = pd["max_neighbors"]
    p.max_boundary_neighbors = pd["max_boundary_neighbors"]
    p.auto_rebuild = pd.get("auto_rebuild", 0)
    p.solver = pd.get("solver", 0)
    p.wcsph_k = pd.get("wcsph_k", 2.8e5)
    p.wcsph_gamma = pd.get("wcsph_gamma", 7.0)
    p.cg_warm_factor = pd.get("cg_warm_factor", 0.0)
    p.separate_div_check = pd.get("separate_div_check", 0)
    p.alpha_max_factor = pd.get("alpha_max_factor", 0.0)
    p.eta_density_max = pd.get("eta_density_max", 0.0)
    p.rigid_coupling = pd.get("rigid_coupling", 0)
    p.rigid_contact = pd.get("rigid_contact", 0)
    return p


def _rigid_array(rigid):
    arr = (sph_rigid_desc * max(1, len(rigid)))()
    for i, r in enumerate(rigid):
        arr[i].mass = r["mass"]
        for a in range(3):
            arr[i].inertia[a] = r["inertia"][a]
            arr[i].com[a] = r["com"][a]
            arr[i].vel[a] = r["vel"][a]
            arr[i].omega[a] = r["omega"][a]
        for a in range(4):
            arr[i].quat[a] = r["quat"][a]
    return arr


def _rigid_dicts(arr, n):
    return [dict(mass=arr[i].mass, inertia=tuple(arr[i].inertia), com=tuple(arr[i].com),
                 quat=tuple(arr[i].quat), vel=tuple(arr[i].vel), omega=tuple(arr[i].omega)) for i in range(n)]


def current_stream_handle() -> Optional[int]:
    """The hipStream_t of torch's current stream on this device (torch owns
    streams; the library borrows one)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def required_bytes(scene, params: Optional[Dict] = None) -> int:
    """sph_required_bytes: the device arena a context of this scene needs."""
    sc = sph_scene()
    sc.n_fluid, sc.n_boundary, sc.n_rigid = scene.n_fluid, scene.n_boundary, len(scene.rigid)
    p = make_params(dict(scene.params if params is None else params))
    out = C.c_int64()
    rc = sph_required_bytes(C.byref(p), C.byref(sc), C.byref(out))
    if rc != SPH_OK:
        raise SphError(rc, sph_last_error(None).decode())
    return out.value


class Simulation:
    """One sph_ctx: create from a scene, build neighbours, step, read state.
    arena: optional device tensor (any dtype, contiguous, on the current
    device, starting 256-byte aligned, as a freshly allocated tensor does)
    lent to the context for all its device buffers; it must hold at least
    required_bytes(scene, params) bytes and is kept alive here."""

    def __init__(self, scene, params: Optional[Dict] = None, stream: Optional[int] = None, arena=None):
        pd = dict(scene.params if params is None else params)
        self.params = pd
        self.nf = scene.n_fluid
        self.nb = scene.n_boundary
        self.nr = len(scene.rigid)
        self._keep = [np.ascontiguousarray(scene.x_fluid, np.float32),
                      np.ascontiguousarray(scene.v_fluid, np.float32),
                      np.ascontiguousarray(scene.x_boundary, np.float32).reshape(-1, 3),
                      np.ascontiguousarray(scene.body_of_boundary, np.int32)]
        self._rigid = _rigid_array(scene.rigid)
        sc = sph_scene()
        sc.n_fluid, sc.n_boundary, sc.n_rigid = self.nf, self.nb, self.nr
        sc.x_fluid, sc.v_fluid, sc.x_boundary, sc.body_of_boundary = (_ptr(a) for a in self._keep)
        sc.rigid = C.cast(self._rigid, C.c_void_p)
        self._arena = arena
        if arena is not None:
            sc.device_arena = C.c_void_p(arena.data_ptr())
            sc.device_arena_bytes = arena.numel() * arena.element_size()
        self._p = make_params(pd)
        ctx = C.c_void_p()
        if stream is None:
            stream = current_stream_handle()
        rc = sph_create(C.byref(self._p), C.byref(sc), C.c_void_p(stream) if stream else None, C.byref(ctx))
        if rc != SPH_OK:
            raise SphError(rc, sph_last_error(None).decode())
        self.ctx = ctx
        self.last_stats = None

    def close(self):
        if getattr(self, "ctx", None):
            sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != SPH_OK:
            raise SphError(rc, sph_last_error(self.ctx).decode())

    def build_neighbors(self):
        self._check(sph_build_neighbors(self.ctx))

    def step(self) -> Dict:
        st = sph_step_stats()
        self._check(sph_step(self.ctx, C.byref(st)))
        self.last_stats = st.as_dict()
        return self.last_stats

    def advance(self) -> Dict:
        """One whole step: the neighbour build and the step (with auto_rebuild
        the step queues the build itself and overlaps its status read with
        the density pass)."""
        if not self.params.get("auto_rebuild", 0):
            self.build_neighbors()
        return self.step()

    def info(self) -> Dict:
        i = sph_info()
        self._check(sph_get_info(self.ctx, C.byref(i)))
        return {k: (tuple(getattr(i, k)) if k in ("grid_n", "origin") else getattr(i, k)) for k, _ in i._fields_}

    def set_forced_iters(self, div: int, dens: int):
        self._check(sph_set_forced_iters(self.ctx, div, dens))

    def read(self, fields=("x", "v", "rho", "alpha", "K", "Kv", "kappa", "accel", "nbr", "psi",
                           "boundary", "rigid")) -> Dict:
        nf, nb, nr = self.nf, self.nb, self.nr
        out: Dict = {}
        hv = sph_host_view()
        mask = 0
        spec3 = {"x": FIELD_X, "v": FIELD_V, "accel": FIELD_ACCEL, "dvisc": FIELD_DVISC}
        spec1 = {"rho": FIELD_RHO, "alpha": FIELD_ALPHA, "K": FIELD_K, "Kv": FIELD_KV, "kappa": FIELD_KAPPA}
        for f, bit in spec3.items():
            if f in fields:
                out[f] = np.zeros((nf, 3), np.float32)
                setattr(hv, f, _ptr(out[f]))
                mask |= bit
        for f, bit in spec1.items():
            if f in fields:
                out[f] = np.zeros(nf, np.float32)
                setattr(hv, f, _ptr(out[f]))
                mask |= bit
        if "nbr" in fields:
            out["nf_count"] = np.zeros(nf, np.int32)
            out["nb_count"] = np.zeros(nf, np.int32)
            hv.n_fluid_nbrs, hv.n_boundary_nbrs = _ptr(out["nf_count"]), _ptr(out["nb_count"])
            mask |= FIELD_NBR
        if "psi" in fields:
            out["psi"] = np.zeros(nb, np.float32)
            hv.psi = _ptr(out["psi"])
            mask |= FIELD_PSI
        if "boundary" in fields:
            out["xb"] = np.zeros((nb, 3), np.float32)
            out["vb"] = np.zeros((nb, 3), np.float32)
            hv.x_boundary, hv.v_boundary = _ptr(out["xb"]), _ptr(out["vb"])
            mask |= FIELD_BOUNDARY
        rig = None
        if "rigid" in fields and nr > 0:
            rig = (sph_rigid_desc * nr)()
            out["force"] = np.zeros((nr, 3))
            out["torque"] = np.zeros((nr, 3))
            hv.rigid = C.cast(rig, C.c_void_p)
            hv.rigid_force, hv.rigid_torque = _ptr(out["force"]), _ptr(out["torque"])
            mask |= FIELD_RIGID
        self._check(sph_read_state(self.ctx, mask, C.byref(hv)))
        if rig is not None:
            out["rigid"] = _rigid_dicts(rig, nr)
        return out

    def write(self, x=None, v=None, K=None, Kv=None, xb=None, vb=None, rigid=None, dvisc=None, rho=None):
        hv = sph_host_view()
        keep = []
        mask = 0

        def put(name, arr, bit, shape):
            nonlocal mask
            if arr is None:
                return
            a = np.ascontiguousarray(arr, np.float32).reshape(shape)
            keep.append(a)
            setattr(hv, name, _ptr(a))
            mask |= bit

        put("x", x, FIELD_X, (self.nf, 3))
        put("v", v, FIELD_V, (self.nf, 3))
        put("K", K, FIELD_K, (self.nf,))
        put("Kv", Kv, FIELD_KV, (self.nf,))
        put("rho", rho, FIELD_RHO, (self.nf,))
        put("dvisc", dvisc, FIELD_DVISC, (self.nf, 3))
        put("x_boundary", xb, FIELD_BOUNDARY, (self.nb, 3))
        put("v_boundary", vb, FIELD_BOUNDARY, (self.nb, 3))
        if rigid is not None:
            arr = _rigid_array(rigid)
            keep.append(arr)
            hv.rigid = C.cast(arr, C.c_void_p)
            mask |= FIELD_RIGID
        self._check(sph_write_state(self.ctx, mask, C.byref(hv)))

    def read_neighbors(self) -> Dict:
        info = self.info()
        ncell = info["grid_n"][0] * info["grid_n"][1] * info["grid_n"][2]
        nf, nb = self.nf, self.nb
        o = {
            "keys_f": np.zeros(nf, np.uint32), "perm_f": np.zeros(nf, np.uint32),
            "start_f": np.zeros(ncell + 1, np.uint32), "counts_f": np.zeros(nf, np.uint32),
            "lists_f": np.zeros(max(1, nf * info["max_neighbors"]), np.uint32),
            "keys_b": np.zeros(nb, np.uint32), "perm_b": np.zeros(nb, np.uint32),
            "start_b": np.zeros(ncell + 1, np.uint32), "counts_b": np.zeros(nf, np.uint32),
            "lists_b": np.zeros(max(1, nf * info["max_boundary_neighbors"]), np.uint32),
        }
        v = sph_nbr_view()
        for k, a in o.items():
            setattr(v, k, _ptr(a))
        v.cap_f, v.cap_b = len(o["lists_f"]), len(o["lists_b"])
        self._check(sph_read_neighbors(self.ctx, C.byref(v)))
        o["lists_f"] = o["lists_f"][: int(o["counts_f"].astype(np.int64).sum())]
        o["lists_b"] = o["lists_b"][: int(o["counts_b"].astype(np.int64).sum())]
        return o

    def set_warm_start(self, mode: int, mlp: Optional["MLP"] = None):
        self._warm_mlp = mlp
        self._check(sph_set_warm_start(self.ctx, mode, mlp.h if mlp is not None else None))

    def enable_trace(self, features, targets, capacity: int):
        """features, targets: device tensors (torch) of [capacity, 5] and [capacity] float32."""
        self._trace = (features, targets)
        fp = None if features is None else C.c_void_p(features.data_ptr())
        tp = None if targets is None else C.c_void_p(targets.data_ptr())
        self._check(sph_enable_trace(self.ctx, fp, tp, capacity))

    def trace_rows(self) -> int:
        n = C.c_int64()
        self._check(sph_trace_rows(self.ctx, C.byref(n)))
        return n.value

    def profile_enable(self, on: bool = True, only: Optional[str] = None):
        """only: record the events of that kernel name alone (None: all)."""
        self._check(sph_profile_only(self.ctx, only.encode() if only else None))
        self._check(sph_profile_enable(self.ctx, 1 if on else 0))

    def profile_read(self, kernel: str) -> Dict:
        n = C.c_int64()
        ms = C.c_double()
        by = C.c_double()
        self._check(sph_profile_read(self.ctx, kernel.encode(), C.byref(n), C.byref(ms), C.byref(by)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}


class MLP:
    """The warm-start MLP on the device (sph_mlp_*); tensors are torch device
    tensors, parameters a float32 numpy vector of MLP_PARAMS entries."""

    def __init__(self, params: np.ndarray, stream: Optional[int] = None):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == MLP_PARAMS
        h = C.c_void_p()
        if stream is None:
            stream = current_stream_handle()
        rc = sph_mlp_create(_ptr(p), C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != SPH_OK:
            raise SphError(rc, sph_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            sph_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != SPH_OK:
            raise SphError(rc, "mlp call failed")

    def params(self) -> np.ndarray:
        p = np.zeros(MLP_PARAMS, np.float32)
        self._check(sph_mlp_get_params(self.h, _ptr(p)))
        return p

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, np.float32)
        self._check(sph_mlp_set_params(self.h, _ptr(p)))

    def forward(self, features, y):
        n = features.shape[0]
        self._check(sph_mlp_forward(self.h, C.c_void_p(features.data_ptr()), C.c_void_p(y.data_ptr()), n))

    def grad(self, features, targets):
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_double()
        self._check(sph_mlp_grad(self.h, C.c_void_p(features.data_ptr()), C.c_void_p(targets.data_ptr()),
                                 features.shape[0], _ptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, features, targets, lr: float) -> float:
        loss = C.c_double()
        self._check(sph_mlp_train_step(self.h, C.c_void_p(features.data_ptr()), C.c_void_p(targets.data_ptr()),
                                       features.shape[0], lr, C.byref(loss)))
        return loss.value
