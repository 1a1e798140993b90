"""Python front of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this module.  It loads ``oracle/liboracle.so`` (plain C,
built by :func:`build`), which shares no code with the HIP library.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source with its independent per-particle loops split over the
# host's cores (OpenMP); every reduction stays sequential in a fixed order, so
# its results equal the single-threaded library's bit for bit
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(force: bool = True, openmp: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction).  openmp=False: one
    thread, the loops run in order (the library the tests use); True: the
    per-particle loops marked in the source run on all cores."""
    out = LIB_OMP if openmp else LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
                               *(["-fopenmp"] if openmp else []), "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, out)
    return out


class Params(C.Structure):
    _fields_ = [
        ("r", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
        ("gravity", C.c_double * 3),
        ("domain_min", C.c_double * 3), ("domain_max", C.c_double * 3),
        ("eta_density", C.c_double), ("eta_divergence", C.c_double),
        ("max_iters", C.c_int32),
        ("dt_max", C.c_double), ("cfl_lambda", C.c_double),
        ("visc_model", C.c_int32), ("visc", C.c_double),
        ("cg_tol", C.c_double), ("cg_max_iters", C.c_int32),
        ("warm_start", C.c_int32),
        ("forced_div", C.c_int32), ("forced_dens", C.c_int32),
        ("n_rigid", C.c_int32),
        ("warm_factor", C.c_double),
        ("solver", C.c_int32), ("wcsph_k", C.c_double), ("wcsph_gamma", C.c_double),
        ("cg_warm_factor", C.c_double),
        ("alpha_max_factor", C.c_double),
        ("eta_density_max", C.c_double),
        ("rigid_coupling", C.c_int32),
        ("rigid_contact", C.c_int32),
    ]


class Rigid(C.Structure):
    _fields_ = [("mass", C.c_double), ("inertia", C.c_double * 3), ("com", C.c_double * 3),
                ("quat", C.c_double * 4), ("vel", C.c_double * 3), ("omega", C.c_double * 3)]


MLP_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double),
                     C.c_void_p)


class In(C.Structure):
    _fields_ = [
        ("nf", C.c_int64), ("nb", C.c_int64),
        ("xf", C.c_void_p), ("vf", C.c_void_p), ("K", C.c_void_p), ("Kv", C.c_void_p),
        ("xb", C.c_void_p), ("vb", C.c_void_p), ("body", C.c_void_p), ("local", C.c_void_p),
        ("rigid", C.c_void_p), ("mlp", MLP_FN), ("mlp_user", C.c_void_p),
        ("brute_force", C.c_int32),
        ("dvisc", C.c_void_p), ("rho_prev", C.c_void_p),
    ]


class Out(C.Structure):
    _fields_ = [
        ("x", C.c_void_p), ("v", C.c_void_p), ("rho", C.c_void_p), ("alpha", C.c_void_p),
        ("K", C.c_void_p), ("Kv", C.c_void_p), ("kappa", C.c_void_p), ("accel", C.c_void_p),
        ("psi", C.c_void_p),
        ("S_x", C.c_void_p), ("S_v", C.c_void_p), ("S_K", C.c_void_p), ("S_Kv", C.c_void_p),
        ("S_kappa", C.c_void_p), ("S_accel", C.c_void_p), ("S_alpha", C.c_void_p),
        ("nf_count", C.c_void_p), ("nb_count", C.c_void_p),
        ("features", C.c_void_p), ("target", C.c_void_p),
        ("S_features", C.c_void_p), ("S_target", C.c_void_p),
        ("xb_new", C.c_void_p), ("vb_new", C.c_void_p), ("rigid_new", C.c_void_p),
        ("force", C.c_void_p), ("torque", C.c_void_p),
        ("S_force", C.c_void_p), ("S_torque", C.c_void_p),
        ("dt", C.c_double),
        ("iters_div", C.c_int32), ("iters_dens", C.c_int32),
        ("converged_div", C.c_int32), ("converged_dens", C.c_int32), ("cg_iters", C.c_int32),
        ("err_div", C.c_double), ("err_dens", C.c_double),
        ("S_err_div", C.c_double), ("S_err_dens", C.c_double), ("cg_resid", C.c_double),
        ("err_div_hist", C.c_double * 128), ("err_dens_hist", C.c_double * 128),
        ("dvisc", C.c_void_p),
        ("err_dens_max", C.c_double), ("err_dens_max_hist", C.c_double * 128),
    ]


class Grid(C.Structure):
    _fields_ = [("cell", C.c_float), ("inv", C.c_float), ("o", C.c_float * 3), ("h2", C.c_float),
                ("n", C.c_int32 * 3)]


_libs = {}
_use_openmp = False


def use_openmp(on: bool) -> None:
    """Route the following calls to the all-cores build (True) or the
    single-threaded one (False, the default)."""
    global _use_openmp
    _use_openmp = bool(on)


def lib():
    key = _use_openmp
    if key not in _libs:
        path = LIB_OMP if key else LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(force=True, openmp=key)
        L = C.CDLL(path)
        L.or_W.restype = C.c_double
        L.or_W.argtypes = [C.c_double, C.c_double]
        L.or_dWdr.restype = C.c_double
        L.or_dWdr.argtypes = [C.c_double, C.c_double]
        L.or_kernel_k.restype = C.c_double
        L.or_kernel_k.argtypes = [C.c_double]
        L.or_grid_make.argtypes = [C.c_double, C.c_void_p, C.c_void_p, C.POINTER(Grid)]
        L.or_cell_keys.argtypes = [C.POINTER(Grid), C.c_void_p, C.c_int64, C.c_void_p]
        L.or_sort_perm.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
        L.or_cell_start.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.or_neighbors_brute.restype = C.c_int64
        L.or_neighbors_brute.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_float, C.c_int32,
                                         C.c_void_p, C.c_void_p, C.c_int64]
        L.or_neighbors_grid.restype = C.c_int64
        L.or_neighbors_grid.argtypes = [C.POINTER(Grid), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p, C.c_void_p, C.c_int64]
        L.or_rigid_local.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.or_boundary_psi.argtypes = [C.POINTER(Params), C.c_void_p, C.c_int64, C.c_void_p]
        L.or_pcisph_factor.restype = C.c_double
        L.or_pcisph_factor.argtypes = [C.POINTER(Params)]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.POINTER(Params), C.POINTER(In), C.POINTER(Out)]
        L.or_visc_dense.argtypes = [C.POINTER(Params), C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p]
        L.or_visc_solve.argtypes = [C.POINTER(Params), C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.or_visc_residual.restype = C.c_double
        L.or_visc_residual.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                                       C.c_void_p, C.c_void_p]
        L.or_density_alpha.argtypes = [C.POINTER(Params), C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
        _libs[key] = L
    return _libs[key]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_params(pd: Dict, forced_div: int = -1, forced_dens: int = -1, n_rigid: int = 0) -> Params:
    p = Params()
    p.r = pd["r"]; p.h = pd["h"]; p.rho0 = pd["rho0"]
    for a in range(3):
        p.gravity[a] = pd["gravity"][a]
        p.domain_min[a] = pd["domain_min"][a]
        p.domain_max[a] = pd["domain_max"][a]
    p.eta_density = pd["eta_density"]; p.eta_divergence = pd["eta_divergence"]
    p.max_iters = pd["max_iters"]
    p.dt_max = pd["dt_max"]; p.cfl_lambda = pd["cfl_lambda"]
    p.visc_model = pd["visc_model"]; p.visc = pd["visc"]
    p.cg_tol = pd["cg_tol"]; p.cg_max_iters = pd["cg_max_iters"]
    p.warm_start = pd["warm_start"]
    p.forced_div = forced_div; p.forced_dens = forced_dens
    p.n_rigid = n_rigid
    p.warm_factor = pd["warm_factor"]
    p.solver = pd.get("solver", 0)
    p.wcsph_k = pd.get("wcsph_k", 2.8e5)
    p.wcsph_gamma = pd.get("wcsph_gamma", 7.0)
    p.cg_warm_factor = pd.get("cg_warm_factor", 0.0)
    p.alpha_max_factor = pd.get("alpha_max_factor", 0.0)
    p.eta_density_max = pd.get("eta_density_max", 0.0)
    p.rigid_coupling = pd.get("rigid_coupling", 0)
    p.rigid_contact = pd.get("rigid_contact", 0)
    return p


# --------------------------------------------------------------------------
# kernel, grid and neighbour pieces
# --------------------------------------------------------------------------
def W(r: float, h: float) -> float:
    return lib().or_W(r, h)


def dWdr(r: float, h: float) -> float:
    return lib().or_dWdr(r, h)


def grid(pd: Dict) -> Grid:
    g = Grid()
    dmin = np.asarray(pd["domain_min"], np.float64)
    dmax = np.asarray(pd["domain_max"], np.float64)
    lib().or_grid_make(pd["h"], _p(dmin), _p(dmax), C.byref(g))
    return g


def cell_keys(g: Grid, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    key = np.empty(len(x), np.uint32)
    lib().or_cell_keys(C.byref(g), _p(x), len(x), _p(key))
    return key


def sort_perm(key: np.ndarray) -> np.ndarray:
    key = np.ascontiguousarray(key, np.uint32)
    perm = np.empty(len(key), np.uint32)
    lib().or_sort_perm(_p(key), len(key), _p(perm))
    return perm


def cell_start(g: Grid, key: np.ndarray, perm: np.ndarray) -> np.ndarray:
    ncell = g.n[0] * g.n[1] * g.n[2]
    st = np.empty(ncell + 1, np.uint32)
    lib().or_cell_start(_p(np.ascontiguousarray(key, np.uint32)), _p(np.ascontiguousarray(perm, np.uint32)),
                        len(key), ncell, _p(st))
    return st


def neighbors(xq_sorted: np.ndarray, xc_sorted: np.ndarray, h2: float, same_set: bool,
              g: Optional[Grid] = None, start: Optional[np.ndarray] = None):
    """CSR (counts, concatenated lists) in sorted-index space; brute force
    when no grid is given."""
    xq = np.ascontiguousarray(xq_sorted, np.float32)
    xc = np.ascontiguousarray(xc_sorted, np.float32)
    counts = np.empty(len(xq), np.uint32)
    cap = 64 * (len(xq) + 1)
    while True:
        out = np.empty(cap, np.uint32)
        if g is None:
            tot = lib().or_neighbors_brute(_p(xq), len(xq), _p(xc), len(xc), C.c_float(h2), int(same_set),
                                           _p(counts), _p(out), cap)
        else:
            tot = lib().or_neighbors_grid(C.byref(g), _p(xq), len(xq), _p(xc), _p(start), int(same_set),
                                          _p(counts), _p(out), cap)
        if tot >= 0:
            return counts, out[:tot].copy()
        cap *= 2


def sorted_neighbor_structure(pd: Dict, x_fluid: np.ndarray, x_boundary: np.ndarray, brute: bool = True):
    """Everything the bit-exact contract covers, as the oracle computes it:
    keys, permutations, cell tables, fluid and boundary neighbour lists."""
    g = grid(pd)
    out = {"grid": g}
    for tag, x in (("f", x_fluid), ("b", x_boundary)):
        key = cell_keys(g, x)
        perm = sort_perm(key)
        out[f"key_{tag}"] = key
        out[f"perm_{tag}"] = perm
        out[f"start_{tag}"] = cell_start(g, key, perm)
        out[f"xs_{tag}"] = np.ascontiguousarray(x[perm])
    xs_f, xs_b = out["xs_f"], out["xs_b"]
    if brute:
        out["nf"] = neighbors(xs_f, xs_f, g.h2, True)
        out["nb"] = neighbors(xs_f, xs_b, g.h2, False)
    else:
        out["nf"] = neighbors(xs_f, xs_f, g.h2, True, g, out["start_f"])
        out["nb"] = neighbors(xs_f, xs_b, g.h2, False, g, out["start_b"])
    return out


def rigid_local(x_boundary: np.ndarray, body: np.ndarray, rigid) -> np.ndarray:
    nb = len(x_boundary)
    local = np.zeros((nb, 3), np.float64)
    rb = (Rigid * max(1, len(rigid)))()
    for i, r in enumerate(rigid):
        _fill_rigid(rb[i], r)
    lib().or_rigid_local(_p(np.ascontiguousarray(x_boundary, np.float32)),
                         _p(np.ascontiguousarray(body, np.int32)), nb, C.cast(rb, C.c_void_p), _p(local))
    return local


def _fill_rigid(dst: Rigid, r: Dict):
    dst.mass = r["mass"]
    for a in range(3):
        dst.inertia[a] = r["inertia"][a]
        dst.com[a] = r["com"][a]
        dst.vel[a] = r["vel"][a]
        dst.omega[a] = r["omega"][a]
    for a in range(4):
        dst.quat[a] = r["quat"][a]


def _rigid_dict(src: Rigid) -> Dict:
    return dict(mass=src.mass, inertia=tuple(src.inertia), com=tuple(src.com), quat=tuple(src.quat),
                vel=tuple(src.vel), omega=tuple(src.omega))


def boundary_psi(pd: Dict, x_boundary: np.ndarray) -> np.ndarray:
    xb = np.ascontiguousarray(x_boundary, np.float32)
    psi = np.empty(len(xb), np.float64)
    p = make_params(pd)
    lib().or_boundary_psi(C.byref(p), _p(xb), len(xb), _p(psi))
    return psi


def density_alpha(pd: Dict, x_fluid: np.ndarray, x_boundary: np.ndarray):
    xf = np.ascontiguousarray(x_fluid, np.float32)
    xb = np.ascontiguousarray(x_boundary, np.float32).reshape(-1, 3)
    rho = np.empty(len(xf)); alpha = np.empty(len(xf)); psi = np.empty(max(1, len(xb)))
    p = make_params(pd)
    lib().or_density_alpha(C.byref(p), _p(xf), len(xf), _p(xb), len(xb), _p(rho), _p(alpha), _p(psi))
    return rho, alpha, psi[:len(xb)]


# --------------------------------------------------------------------------
# the step
# --------------------------------------------------------------------------
class State:
    """FP32 state the step consumes (mirrors what the GPU carries)."""

    def __init__(self, scene, local=None):
        self.params = dict(scene.params)
        self.x = np.ascontiguousarray(scene.x_fluid, np.float32).copy()
        self.v = np.ascontiguousarray(scene.v_fluid, np.float32).copy()
        n = len(self.x)
        self.K = np.zeros(n, np.float32)
        self.Kv = np.zeros(n, np.float32)
        self.xb = np.ascontiguousarray(scene.x_boundary, np.float32).copy()
        self.body = np.ascontiguousarray(scene.body_of_boundary, np.int32).copy()
        self.rigid = [dict(r) for r in scene.rigid]
        self.local = rigid_local(self.xb, self.body, self.rigid) if local is None else local
        self.vb = np.zeros_like(self.xb)
        self.dvisc = np.zeros((n, 3), np.float32)   # previous implicit-viscosity correction
        self.rho_prev = np.full(n, np.float32(self.params["rho0"]), np.float32)   # previous step's density


def pcisph_factor(pd: Dict) -> float:
    """PCISPH stiffness factor c of kappa_i = (rho*_i - rho0) c / (rho_i dt^2)."""
    p = make_params(pd)
    return float(lib().or_pcisph_factor(C.byref(p)))


def step(state: State, forced_div: int = -1, forced_dens: int = -1, brute: Optional[bool] = None,
         mlp=None, want_features: bool = False, params: Optional[Dict] = None) -> Dict:
    """One oracle DFSPH step from ``state`` (not modified); returns all
    outputs (FP64 fields in id order, scales, stats)."""
    pd = dict(state.params if params is None else params)
    nf, nb = len(state.x), len(state.xb)
    nr = len(state.rigid)
    p = make_params(pd, forced_div, forced_dens, nr)
    if brute is None:
        brute = (nf + nb) <= 6000
    xf = np.ascontiguousarray(state.x, np.float32)
    vf = np.ascontiguousarray(state.v, np.float32)
    K = np.ascontiguousarray(state.K, np.float32)
    Kv = np.ascontiguousarray(state.Kv, np.float32)
    xb = np.ascontiguousarray(state.xb, np.float32).reshape(-1, 3)
    vb = np.ascontiguousarray(state.vb, np.float32).reshape(-1, 3)
    body = np.ascontiguousarray(state.body, np.int32)
    local = np.ascontiguousarray(state.local, np.float64).reshape(-1, 3)
    rb = (Rigid * max(1, nr))()
    for i, r in enumerate(state.rigid):
        _fill_rigid(rb[i], r)

    ci = In()
    ci.nf, ci.nb = nf, nb
    ci.xf, ci.vf, ci.K, ci.Kv = _p(xf), _p(vf), _p(K), _p(Kv)
    ci.xb, ci.vb, ci.body, ci.local = _p(xb), _p(vb), _p(body), _p(local)
    ci.rigid = C.cast(rb, C.c_void_p)
    ci.brute_force = int(bool(brute))
    dv = np.ascontiguousarray(getattr(state, "dvisc", np.zeros((nf, 3))), np.float32).reshape(nf, 3)
    ci.dvisc = _p(dv)
    rp = np.ascontiguousarray(getattr(state, "rho_prev", np.full(nf, pd["rho0"])), np.float32).reshape(nf)
    ci.rho_prev = _p(rp)
    keep = []
    if mlp is not None:
        def _cb(fp, sp, n, yp, user):
            F = np.ctypeslib.as_array(fp, shape=(n, 5)).copy()
            SF = np.ctypeslib.as_array(sp, shape=(n, 5)).copy()
            res = mlp(F, SF)
            y, err = (res if isinstance(res, tuple) else (res, np.zeros(n)))
            out = np.ctypeslib.as_array(yp, shape=(2 * n,))
            out[:n] = np.asarray(y, np.float64).reshape(n)
            out[n:] = np.asarray(err, np.float64).reshape(n)
        cb = MLP_FN(_cb)
        keep.append(cb)
        ci.mlp = cb
    else:
        ci.mlp = MLP_FN()

    o = {k: np.zeros((nf, 3)) for k in ("x", "v", "accel", "S_x", "S_v", "S_accel", "dvisc")}
    for k in ("rho", "alpha", "K", "Kv", "kappa", "S_K", "S_Kv", "S_kappa", "S_alpha"):
        o[k] = np.zeros(nf)
    o["psi"] = np.zeros(max(1, nb))
    o["nf_count"] = np.zeros(nf, np.int32)
    o["nb_count"] = np.zeros(nf, np.int32)
    o["xb_new"] = np.zeros((max(1, nb), 3), np.float32)
    o["vb_new"] = np.zeros((max(1, nb), 3), np.float32)
    o["force"] = np.zeros((max(1, nr), 3))
    o["torque"] = np.zeros((max(1, nr), 3))
    o["S_force"] = np.zeros((max(1, nr), 3))
    o["S_torque"] = np.zeros((max(1, nr), 3))
    feats = want_features or pd["warm_start"] == 2
    if want_features:
        o["features"] = np.zeros((nf, 5))
        o["target"] = np.zeros(nf)
        o["S_features"] = np.zeros((nf, 5))
        o["S_target"] = np.zeros(nf)
    rnew = (Rigid * max(1, nr))()
    co = Out()
    for k, a in o.items():
        setattr(co, k, _p(a))
    co.rigid_new = C.cast(rnew, C.c_void_p)
    if not want_features:
        co.features = None
        co.target = None
        co.S_features = None
        co.S_target = None
    rc = lib().or_step(C.byref(p), C.byref(ci), C.byref(co))
    if rc != 0:
        raise RuntimeError(f"or_step failed: {rc}")
    del feats
    o["psi"] = o["psi"][:nb]
    o["xb_new"] = o["xb_new"][:nb]
    o["vb_new"] = o["vb_new"][:nb]
    for k in ("force", "torque", "S_force", "S_torque"):
        o[k] = o[k][:nr]
    o["rigid_new"] = [_rigid_dict(rnew[i]) for i in range(nr)]
    for k in ("dt", "iters_div", "iters_dens", "converged_div", "converged_dens", "cg_iters", "err_div",
              "err_dens", "S_err_div", "S_err_dens", "cg_resid", "err_dens_max"):
        o[k] = getattr(co, k)
    o["err_div_hist"] = np.array(co.err_div_hist[:min(128, o["iters_div"] + 1)])
    o["err_dens_hist"] = np.array(co.err_dens_hist[:min(128, o["iters_dens"] + 1)])
    o["err_dens_max_hist"] = np.array(co.err_dens_max_hist[:min(128, o["iters_dens"] + 1)])
    return o


def advance(state: State, out: Dict) -> State:
    """The next step's FP32 state from a step's outputs (the GPU carries
    FP32, so the oracle's multi-step runs round to FP32 in between)."""
    s = State.__new__(State)
    s.params = state.params
    s.x = out["x"].astype(np.float32)
    s.v = out["v"].astype(np.float32)
    s.K = out["K"].astype(np.float32)
    s.Kv = out["Kv"].astype(np.float32)
    s.xb = out["xb_new"].astype(np.float32)
    s.vb = out["vb_new"].astype(np.float32)
    s.body = state.body
    s.local = state.local
    s.rigid = out["rigid_new"]
    s.dvisc = out["dvisc"].astype(np.float32)
    s.rho_prev = out["rho"].astype(np.float32)
    return s


# --------------------------------------------------------------------------
# implicit viscosity pieces
# --------------------------------------------------------------------------
def visc_dense(pd: Dict, x_fluid: np.ndarray, dt: float):
    xf = np.ascontiguousarray(x_fluid, np.float32)
    n3 = 3 * len(xf)
    M = np.zeros((n3, n3))
    rho = np.zeros(len(xf))
    lib().or_visc_dense(C.byref(make_params(pd)), _p(xf), len(xf), dt, _p(M), _p(rho))
    return M, rho


def visc_solve(pd: Dict, x_fluid: np.ndarray, dt: float, b: np.ndarray):
    xf = np.ascontiguousarray(x_fluid, np.float32)
    b = np.ascontiguousarray(b, np.float64).reshape(-1)
    x = np.zeros_like(b)
    it = C.c_int32()
    res = C.c_double()
    lib().or_visc_solve(C.byref(make_params(pd)), _p(xf), len(xf), dt, _p(b), _p(x), C.byref(it), C.byref(res))
    return x.reshape(-1, 3), it.value, res.value


def visc_residual(pd: Dict, x_fluid: np.ndarray, rho: np.ndarray, dt: float, b: np.ndarray, x: np.ndarray) -> float:
    xf = np.ascontiguousarray(x_fluid, np.float32)
    b = np.ascontiguousarray(b, np.float64).reshape(-1)
    x = np.ascontiguousarray(x, np.float64).reshape(-1)
    rho = np.ascontiguousarray(rho, np.float64)
    return lib().or_visc_residual(C.byref(make_params(pd)), _p(xf), _p(rho), len(xf), dt, _p(b), _p(x))
