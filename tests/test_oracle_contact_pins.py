"""Pins of the oracle's rigid contact (frictionless, no restitution; the
bodies' sample points are their contact geometry; projected Gauss-Seidel on
normal impulses at the step's end).  The paper takes rigid dynamics and
contact from a physics engine (Sec. 4.2); what is pinned here is what the
model fixes: a body at rest on the floor takes exactly its weight, two equal
boxes meeting head-on stop one sampling spacing apart, every impulse pair
keeps linear and angular momentum, a projection onto non-approaching
velocities loses kinetic energy, and a dropped body does not sink into the
floor."""

import numpy as np

from oracle import oracle as O
from paper_2403_11156_amd import scenes

R_ = 0.01
S_ = 2.0 * R_


def setup_module(_):
    O.build(force=False)


def _box(com, quat=(1.0, 0.0, 0.0, 0.0), n=7, dens=500.0):
    size = (n - 1) * S_
    pts = scenes.shell((n, n, n), (-size / 2,) * 3, S_)
    mass = dens * size ** 3
    return dict(local_points=pts, mass=mass, inertia=(mass * size * size / 6.0,) * 3, com=tuple(com),
                quat=tuple(quat), kind="box", size=size)


def _scene(bodies, vels=None, omegas=None, gravity=(0.0, -9.81, 0.0), tank=(0.6, 0.6, 0.6), contact=1):
    # bodies and the tank, no fluid
    sc = scenes.make_block_scene("contact", R_, (0, 0, 0), tank, (0, 0, 0), (R_, R_, R_), seed=5, steps=1,
                                 bodies=bodies, gravity=gravity, cfl_lambda=0.0, dt_max=1e-3,
                                 rigid_contact=contact)
    for i in range(len(bodies)):
        sc.rigid[i] = dict(sc.rigid[i], vel=tuple((vels or {}).get(i, (0.0, 0.0, 0.0))),
                           omega=tuple((omegas or {}).get(i, (0.0, 0.0, 0.0))))
    return sc


def _points(sc, state, b):
    loc = state.local[state.body == b]
    R = scenes.quat_to_matrix(state.rigid[b]["quat"])
    return loc @ R.T + np.asarray(state.rigid[b]["com"])


def _energy(state, g=9.81):
    e = 0.0
    for s in state.rigid:
        R = scenes.quat_to_matrix(s["quat"])
        Iw = R @ np.diag(s["inertia"]) @ R.T
        v = np.asarray(s["vel"])
        w = np.asarray(s["omega"])
        e += 0.5 * s["mass"] * v @ v + 0.5 * w @ Iw @ w + s["mass"] * g * s["com"][1]
    return e


def test_box_at_rest_on_the_floor_takes_exactly_its_weight():
    # bottom face on the plane min + r (its sample points as the oracle holds
    # them, after their FP32 rounding): every step the contact impulses sum to
    # M g dt, so the box neither moves nor turns
    b = _box((0.3, R_ + 3 * S_, 0.3))
    sc = _scene([b])
    st = O.State(sc)
    lift = R_ - _points(sc, st, 0)[:, 1].min()
    sc.rigid[0] = dict(sc.rigid[0], com=(0.3, R_ + 3 * S_ + lift, 0.3))
    st.rigid = sc.rigid
    c0 = np.asarray(sc.rigid[0]["com"])
    for k in range(50):
        out = O.step(st, brute=False)
        st = O.advance(st, out)
        s = st.rigid[0]
        assert np.abs(s["vel"]).max() < 1e-6 * 9.81 * out["dt"], (k, s["vel"])
        assert np.abs(s["omega"]).max() < 1e-6, (k, s["omega"])
    assert np.abs(np.asarray(st.rigid[0]["com"]) - c0).max() < 1e-9


def test_equal_boxes_meeting_head_on_stop_one_spacing_apart():
    # no gravity, +-1 m/s along x, faces aligned: without restitution both
    # stop, and their facing sample-point layers end exactly s apart
    a = _box((0.22, 0.3, 0.3))
    b = _box((0.38, 0.3, 0.3))
    sc = _scene([a, b], vels={0: (1.0, 0.0, 0.0), 1: (-1.0, 0.0, 0.0)}, gravity=(0.0, 0.0, 0.0))
    st = O.State(sc)
    M = a["mass"]
    for k in range(40):
        out = O.step(st, brute=False)
        st = O.advance(st, out)
        p = M * (np.asarray(st.rigid[0]["vel"]) + np.asarray(st.rigid[1]["vel"]))
        assert np.abs(p).max() < 1e-12 * M, (k, p)
    gap = _points(sc, st, 1)[:, 0].min() - _points(sc, st, 0)[:, 0].max()
    assert abs(gap - S_) < 1e-9, gap
    for s in st.rigid:
        assert np.abs(s["vel"]).max() < 1e-9 and np.abs(s["omega"]).max() < 1e-9, s


def test_oblique_impact_keeps_momentum_and_loses_energy():
    # unequal, turned boxes, one struck off its centre: on the step of impact
    # the impulse pairs change neither linear nor angular momentum (about the
    # origin, at the step's starting pose), and the kinetic energy drops
    a = _box((0.15, 0.28, 0.3), quat=scenes._random_quat(0.3, 0.6, 0.1))
    b = _box((0.42, 0.32, 0.31), quat=scenes._random_quat(0.8, 0.2, 0.7), dens=900.0)
    sc = _scene([a, b], vels={0: (1.5, 0.0, 0.0), 1: (-0.5, 0.0, 0.0)}, gravity=(0.0, 0.0, 0.0))
    st = O.State(sc)
    hit = False
    for k in range(40):
        out = O.step(st, brute=False)
        before, after = st.rigid, out["rigid_new"]
        turned = any(np.abs(s["omega"]).max() > 0 for s in after)
        if turned and not hit:
            hit = True
            P0 = sum(s["mass"] * np.asarray(s["vel"]) for s in before)
            P1 = sum(s["mass"] * np.asarray(s["vel"]) for s in after)
            np.testing.assert_allclose(P1, P0, rtol=0, atol=1e-12 * np.abs(P0).max())
            L0 = np.zeros(3)
            L1 = np.zeros(3)
            E0 = E1 = 0.0
            for s0, s1 in zip(before, after):
                R = scenes.quat_to_matrix(s0["quat"])
                Iw = R @ np.diag(s0["inertia"]) @ R.T
                c = np.asarray(s0["com"])
                L0 += s0["mass"] * np.cross(c, s0["vel"]) + Iw @ np.asarray(s0["omega"])
                L1 += s1["mass"] * np.cross(c, s1["vel"]) + Iw @ np.asarray(s1["omega"])
                E0 += 0.5 * s0["mass"] * np.dot(s0["vel"], s0["vel"])
                E1 += 0.5 * s1["mass"] * np.dot(s1["vel"], s1["vel"]) + 0.5 * np.asarray(s1["omega"]) @ Iw @ s1["omega"]
            np.testing.assert_allclose(L1, L0, rtol=0, atol=1e-12 * np.abs(L0).max())
            assert E1 < E0, (E0, E1)
        st = O.advance(st, out)
    assert hit


def test_dropped_box_lands_without_sinking_and_comes_to_rest():
    # a turned box released 5 cm above the floor: its lowest sample point
    # never goes below the plane min + r by more than a thousandth of s, the
    # total energy never rises, and it ends at rest
    b = _box((0.3, 0.3, 0.3), quat=scenes._random_quat(0.4, 0.3, 0.9))
    sc = _scene([b])
    st = O.State(sc)
    lift = R_ + 0.05 - _points(sc, st, 0)[:, 1].min()
    sc = _scene([dict(b, com=(0.3, 0.3 + lift, 0.3))])
    st = O.State(sc)
    e = _energy(st)
    M = b["mass"]
    low = []
    for k in range(600):
        out = O.step(st, brute=False)
        st = O.advance(st, out)
        low.append(_points(sc, st, 0)[:, 1].min() - R_)
        e1 = _energy(st)
        assert e1 <= e + 1e-3 * M * 9.81 * S_, (k, e, e1)
        e = e1
    assert min(low) > -1e-3 * S_, min(low)
    assert np.abs(st.rigid[0]["vel"]).max() < 1e-3 and np.abs(st.rigid[0]["omega"]).max() < 1e-2


def test_without_contact_the_boxes_pass_through_each_other():
    a = _box((0.22, 0.3, 0.3))
    b = _box((0.38, 0.3, 0.3))
    sc = _scene([a, b], vels={0: (1.0, 0.0, 0.0), 1: (-1.0, 0.0, 0.0)}, gravity=(0.0, 0.0, 0.0), contact=0)
    st = O.State(sc)
    for _ in range(40):
        st = O.advance(st, O.step(st))
    assert st.rigid[0]["vel"][0] == 1.0 and st.rigid[1]["vel"][0] == -1.0
