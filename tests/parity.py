"""Shared helpers of the GPU-vs-oracle tests (not a test module)."""

import numpy as np

from oracle import oracle as O

# Single-step fields: |f_gpu - f_ref| <= REL * (|f_ref| + S_f) + ULP_MIN, S_f the
# oracle's running error scale (zero for rho and alpha, which are sums of
# positive terms).  ULP_MIN covers FP32's subnormal range: the device keeps
# its fields in FP32, so a value that has decayed below FP32's normal range
# (an isolated particle's warm-started K or Kv shrinks by the warm factor
# every step) is rounded to the subnormal spacing 2^-149 whatever its
# relative scale, and the divergence start carries Kv as stiffness over
# density (x.w) and multiplies it back by the density, up to ~2000 kg/m^3 =
# 2^11: an absolute rounding of up to 2^-149 * 2^11.
REL = 1e-5
ULP_MIN = 2.0 ** -138


def ratio(gpu, ref, scale=None):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    s = np.abs(ref) if scale is None else np.abs(ref) + np.asarray(scale, np.float64)
    tol = REL * s + ULP_MIN
    d = np.abs(gpu - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(tol > 0, d / np.where(tol > 0, tol, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def oracle_state_from_gpu(sim, scene, local):
    """Re-anchor: the oracle's FP32 input state is exactly the GPU's state."""
    g = sim.read(("x", "v", "K", "Kv", "rho", "boundary", "rigid", "dvisc"))
    st = O.State.__new__(O.State)
    st.params = dict(sim.params)
    st.x, st.v = g["x"], g["v"]
    st.K, st.Kv = g["K"], g["Kv"]
    st.xb, st.vb = g["xb"], g["vb"]
    st.body = np.ascontiguousarray(scene.body_of_boundary, np.int32)
    st.local = local
    st.rigid = g.get("rigid", [])
    st.dvisc = g["dvisc"]
    st.rho_prev = g["rho"]   # the previous step's density (the divergence warm start's)
    return st


def compare_step(g, ref, stats):
    """Max tolerance ratio per field (<= 1 passes)."""
    out = {
        "rho": ratio(g["rho"], ref["rho"]),
        "alpha": ratio(g["alpha"], ref["alpha"], ref["S_alpha"]),
        "x": ratio(g["x"], ref["x"], ref["S_x"]),
        "v": ratio(g["v"], ref["v"], ref["S_v"]),
        "K": ratio(g["K"], ref["K"], ref["S_K"]),
        "Kv": ratio(g["Kv"], ref["Kv"], ref["S_Kv"]),
        "kappa": ratio(g["kappa"], ref["kappa"], ref["S_kappa"]),
        "accel": ratio(g["accel"], ref["accel"], ref["S_accel"]),
    }
    assert stats["dt"] == ref["dt"], (stats["dt"], ref["dt"])
    return out
