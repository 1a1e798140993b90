"""Pins of the oracle's strong (interlinked) rigid-fluid coupling (our
reading of Sec. 6's future work: every pressure pass moves the bodies at once
and the next pass sees their new boundary velocities)."""

import numpy as np

from oracle import oracle as O
from paper_2403_11156_amd import scenes


def setup_module(_):
    O.build(force=False)


def _scene(mass_scale=1.0, walls=True, centre=(0.2, 0.16, 0.2), height=0.3, **kw):
    r = 0.01
    bodies = scenes.small_bodies(r, 4, [centre])
    for b in bodies:
        b["mass"] *= mass_scale
        b["inertia"] = tuple(i * mass_scale for i in b["inertia"])
    sc = scenes.make_block_scene("coupled", r, (0, 0, 0), (0.4, height, 0.4), (12, 9, 12), (0.08, 0.05, 0.08),
                                 seed=21, steps=1, bodies=bodies, **kw)
    if not walls:
        keep = sc.body_of_boundary >= 0
        sc.x_boundary = np.ascontiguousarray(sc.x_boundary[keep])
        sc.body_of_boundary = np.ascontiguousarray(sc.body_of_boundary[keep])
    return sc


def _state(sc, vel=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0)):
    sc.rigid[0] = dict(sc.rigid[0], vel=vel, omega=omega)
    st = O.State(sc)
    st.v = np.random.default_rng(3).normal(0, 0.3, st.v.shape).astype(np.float32)
    # boundary velocities of the body at the start of the step
    R = scenes.quat_to_matrix(sc.rigid[0]["quat"])
    on = st.body == 0
    rr = st.xb[on].astype(np.float64) - np.asarray(sc.rigid[0]["com"])
    st.vb[on] = (np.asarray(vel) + np.cross(np.asarray(omega), rr)).astype(np.float32)
    del R
    return st


def test_heavy_body_without_gravity_is_the_weak_coupling():
    # a body a trillion times heavier does not move during the step, so with
    # gravity off every pass sees the same boundary velocities as the weak
    # coupling: the same fluid bits, the same reaction up to summation order
    sc = _scene(mass_scale=1e12, gravity=(0.0, 0.0, 0.0))
    st = _state(sc, vel=(0.1, -0.2, 0.05), omega=(0.5, 0.0, -0.3))
    weak = O.step(st, forced_div=2, forced_dens=3)
    strong = O.step(st, forced_div=2, forced_dens=3, params=dict(st.params, rigid_coupling=1))
    for k in ("x", "v", "rho", "K", "Kv"):
        assert np.array_equal(weak[k], strong[k]), k
    assert np.abs(weak["force"]).max() > 0
    np.testing.assert_allclose(strong["force"], weak["force"], rtol=1e-10)
    np.testing.assert_allclose(strong["torque"], weak["torque"], rtol=1e-10, atol=1e-12 * np.abs(weak["torque"]).max())


def test_strong_coupling_conserves_momentum_pass_by_pass():
    # no static walls and no gravity: every pass's impulse on the fluid is
    # minus the impulse on the body (Eq. 14), so fluid plus body keep their
    # total momentum; and the body has moved during the step, unlike a body
    # whose velocity is held (weak coupling), so the fluid ends differently
    sc = _scene(walls=False, gravity=(0.0, 0.0, 0.0), visc_model=0)
    st = _state(sc, vel=(0.0, -0.3, 0.0))
    pd = dict(st.params, rigid_coupling=1)
    out = O.step(st, forced_div=3, forced_dens=4, params=pd)
    m = 1000.0 * (2 * 0.01) ** 3
    M = sc.rigid[0]["mass"]
    dp = m * (out["v"] - st.v.astype(np.float64)).sum(axis=0) + \
        M * (np.asarray(out["rigid_new"][0]["vel"]) - np.asarray(sc.rigid[0]["vel"]))
    scale = m * np.abs(out["v"] - st.v).sum()
    assert np.abs(out["force"][0]).max() > 0 and scale > 0
    assert np.abs(dp).max() < 1e-9 * scale
    # the body's velocity change is the step's summed reaction
    np.testing.assert_allclose(np.asarray(out["rigid_new"][0]["vel"]) - np.asarray(sc.rigid[0]["vel"]),
                               out["dt"] * out["force"][0] / M, rtol=1e-9, atol=1e-15)
    weak = O.step(st, forced_div=3, forced_dens=4, params=dict(pd, rigid_coupling=0))
    assert not np.array_equal(weak["v"], out["v"])


def test_strong_coupling_gravity_reaches_the_body_between_the_solves():
    # a body far from any fluid falls freely: V_new = V + dt g exactly,
    # whichever coupling, and the boundary velocities of the next step follow
    sc = _scene(gravity=(0.0, -9.81, 0.0), centre=(0.2, 0.35, 0.2), height=0.5)
    sc.x_fluid = np.ascontiguousarray(sc.x_fluid[sc.x_fluid[:, 1] < 0.1])
    sc.v_fluid = np.zeros_like(sc.x_fluid)
    st = O.State(sc)
    for coupling in (0, 1):
        out = O.step(st, params=dict(st.params, rigid_coupling=coupling))
        assert np.all(out["force"] == 0.0)
        np.testing.assert_allclose(out["rigid_new"][0]["vel"], (0.0, -9.81 * out["dt"], 0.0), rtol=1e-14, atol=0)
