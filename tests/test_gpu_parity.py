"""HIP path against the FP64 oracle, through the C ABI, on the device.

Bit-exact: cell keys, permutation, cell table, neighbour counts and lists, dt.
Fields: within 1e-5 of the oracle relative to |f| plus its running error
scale, with the oracle run for the GPU's iteration counts (the stop decision
itself is checked separately).
"""

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_11156_amd import scenes

from tests.parity import compare_step, oracle_state_from_gpu, ratio

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sph():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_11156_amd import sph as mod
    O.build(force=False)
    return mod


def _small_with_bodies():
    r = 0.01
    bodies = scenes.small_bodies(r, 4, [(0.22, 0.12, 0.2)])
    return scenes.make_block_scene("small+body", r, (0, 0, 0), (0.4, 0.3, 0.4), (9, 7, 8), (0.012, 0.012, 0.012),
                                   seed=21, steps=1, bodies=bodies, cfl_lambda=0.4, dt_max=1e-3)


def _adversarial_scene():
    rng = np.random.default_rng(17)
    sc = scenes.small_scene(1, 1, 1, tank=(0.3, 0.2, 0.25))
    pd = sc.params
    g = O.grid(pd)
    lo, hi = np.array(pd["domain_min"]), np.array(pd["domain_max"])
    n = 3000
    x = lo + (hi - lo) * rng.random((n, 3))
    x[:300] = np.floor((x[:300] - np.array(g.o)) / g.cell) * g.cell + np.array(g.o)   # on cell faces
    x[300:320] = lo - 0.3 * rng.random((20, 3))                                         # escaped
    x[320:340] = hi + 0.3 * rng.random((20, 3))
    x[340:360] = x[360:380]                                                             # coincident
    x = x.astype(np.float32)
    x[380:400] = x[400:420]
    x[380:400, 0] = x[400:420, 0] + np.float32(pd["h"])                                 # FP32 distance h
    xb = (lo + (hi - lo) * rng.random((1500, 3))).astype(np.float32)
    sc.x_fluid = x
    sc.v_fluid = np.zeros_like(x)
    sc.x_boundary = xb
    sc.body_of_boundary = np.full(len(xb), -1, np.int32)
    sc.params = dict(pd, max_neighbors=96, max_boundary_neighbors=96)
    return sc


NBR_SCENES = {
    "small": lambda: scenes.small_scene(6, 5, 4),
    "c1": lambda: scenes.scene("c1"),
    "bodies": _small_with_bodies,
    "adversarial": _adversarial_scene,
}


@pytest.mark.parametrize("name", list(NBR_SCENES))
def test_neighbour_structure_bit_exact(sph, name):
    sc = NBR_SCENES[name]()
    print(f"[nbr] {name} nf={sc.n_fluid} nb={sc.n_boundary}", flush=True)
    sim = sph.Simulation(sc)
    sim.build_neighbors()
    g = sim.read_neighbors()
    ref = O.sorted_neighbor_structure(sc.params, sc.x_fluid, sc.x_boundary, brute=sc.n_fluid <= 4000)
    np.testing.assert_array_equal(g["perm_f"], ref["perm_f"])
    np.testing.assert_array_equal(g["keys_f"], ref["key_f"][ref["perm_f"]])
    np.testing.assert_array_equal(g["start_f"], ref["start_f"])
    np.testing.assert_array_equal(g["perm_b"], ref["perm_b"])
    np.testing.assert_array_equal(g["keys_b"], ref["key_b"][ref["perm_b"]])
    np.testing.assert_array_equal(g["start_b"], ref["start_b"])
    np.testing.assert_array_equal(g["counts_f"], ref["nf"][0])
    np.testing.assert_array_equal(g["lists_f"], ref["nf"][1])
    np.testing.assert_array_equal(g["counts_b"], ref["nb"][0])
    np.testing.assert_array_equal(g["lists_b"], ref["nb"][1])
    sim.close()


STEP_SCENES = {
    "small_prev": lambda: scenes.small_scene(6, 5, 4),
    "small_zero": lambda: scenes.small_scene(7, 6, 5, warm_start=0, cfl_lambda=0.0, dt_max=4e-4),
    "laplacian": lambda: scenes.small_scene(8, 6, 5, visc_model=scenes.VISC_LAPLACIAN, visc=0.05),
    "bodies": _small_with_bodies,
    "c1": lambda: scenes.scene("c1"),
}


@pytest.mark.parametrize("name", list(STEP_SCENES))
def test_single_step_fields(sph, name):
    sc = STEP_SCENES[name]()
    print(f"[step] {name} nf={sc.n_fluid} nb={sc.n_boundary}", flush=True)
    sim = sph.Simulation(sc)
    local = O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid)
    sim.build_neighbors()
    st = sim.step()
    g = sim.read()
    ref = O.step(O.State(sc, local), forced_div=st["iters_div"], forced_dens=st["iters_dens"])
    r = compare_step(g, ref, st)
    print(name, st["iters_div"], st["iters_dens"], {k: f"{v:.3g}" for k, v in r.items()}, flush=True)
    for k, v in r.items():
        assert v <= 1.0, (k, v)
    np.testing.assert_array_equal(g["nf_count"], ref["nf_count"])
    np.testing.assert_array_equal(g["nb_count"], ref["nb_count"])
    assert ratio(g["psi"], ref["psi"]) <= 1.0
    if sc.rigid:
        assert ratio(g["force"], ref["force"], ref["S_force"]) <= 1.0
        assert ratio(g["torque"], ref["torque"], ref["S_torque"]) <= 1.0
        for a, b in zip(g["rigid"], ref["rigid_new"]):
            np.testing.assert_allclose(a["com"], b["com"], rtol=0, atol=1e-9)
            np.testing.assert_allclose(a["vel"], b["vel"], rtol=1e-6, atol=1e-9)
    sim.close()


def test_stop_rule_and_iteration_counts(sph):
    sc = scenes.scene("c1")
    sim = sph.Simulation(sc)
    local = O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid)
    p = sc.params
    for k in range(8):
        sim.build_neighbors()
        state = oracle_state_from_gpu(sim, sc, local)
        st = sim.step()
        assert st["err_div"] <= p["eta_divergence"] or st["iters_div"] == p["max_iters"]
        assert st["err_dens"] <= p["eta_density"] or st["iters_dens"] == p["max_iters"]
        ref = O.step(state)
        # the oracle takes the same decisions unless the error it tested at
        # the deciding iteration, min(gpu, oracle), lies within 1e-5 S_err of
        # eta (S_err the oracle's running error scale of that mean): then the
        # two stop one iteration apart
        # (for the density solve the bound on the largest compression may be
        # the deciding test instead, with the same band)
        for which in ("div", "dens"):
            gi, oi = st["iters_" + which], ref["iters_" + which]
            if gi != oi:
                hist = ref[f"err_{which}_hist"]
                eta = p["eta_divergence" if which == "div" else "eta_density"]
                band = 1e-5 * ref["S_err_" + which]
                l = min(gi, oi)
                near = abs(hist[l] - eta) <= band
                if which == "dens" and p.get("eta_density_max", 0.0) > 0.0:
                    near = near or abs(ref["err_dens_max_hist"][l] - p["eta_density_max"]) <= band
                assert abs(gi - oi) == 1 and near, (k, which, gi, oi, hist, band)


def test_reanchored_steps_c1(sph):
    # the 8k dam break over its 100 steps: at steps 0, 1, 10, 50 and 100 the
    # oracle takes the device's state and the two steps are compared
    sc = scenes.scene("c1")
    sim = sph.Simulation(sc)
    local = O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid)
    worst = {}
    for k in range(101):
        sim.build_neighbors()
        due = k in (0, 1, 10, 50, 100)
        state = oracle_state_from_gpu(sim, sc, local) if due else None
        st = sim.step()
        if due:
            g = sim.read()
            ref = O.step(state, forced_div=st["iters_div"], forced_dens=st["iters_dens"], brute=False)
            r = compare_step(g, ref, st)
            for f, v in r.items():
                worst[f] = max(worst.get(f, 0.0), v)
    print("worst ratios", worst, flush=True)
    for f, v in worst.items():
        assert v <= 1.0, (f, v)


def test_deterministic(sph):
    outs = []
    for _ in range(2):
        sc = scenes.scene("c1")
        sim = sph.Simulation(sc)
        for _ in range(3):
            sim.advance()
        outs.append(sim.read(("x", "v", "K", "Kv")))
        sim.close()
    for f in outs[0]:
        assert np.array_equal(outs[0][f], outs[1][f]), f


@pytest.mark.parametrize("name", ["c1", "bodies"])
def test_auto_rebuild_matches_explicit_build(sph, name):
    # with auto_rebuild the step queues the next step's sort and build at its
    # end and reads their status after the next density pass: the same
    # computation, bit for bit, as build + step, and every field read back
    # after every step (also those the queued sort has not reordered) agrees
    fields = ("x", "v", "rho", "alpha", "K", "Kv", "kappa", "accel", "nbr", "rigid")
    outs = []
    for auto in (0, 1):
        sc = scenes.scene("c1") if name == "c1" else _small_with_bodies()
        sim = sph.Simulation(sc, params=dict(sc.params, auto_rebuild=auto))
        stats, reads = [], []
        for _ in range(4):
            stats.append(sim.advance())
            reads.append(sim.read(fields))
        outs.append((reads, stats))
        sim.close()
    for k, (ra, rb) in enumerate(zip(outs[0][0], outs[1][0])):
        for f in ("x", "v", "rho", "alpha", "K", "Kv", "kappa", "accel", "nf_count", "nb_count"):
            assert np.array_equal(ra[f], rb[f]), (k, f)
    for a, b in zip(outs[0][1], outs[1][1]):
        for k in ("dt", "iters_div", "iters_dens", "nbr_min", "nbr_max", "nbr_mean"):
            assert a[k] == b[k], k


def test_auto_rebuild_capacity_error(sph):
    sc = scenes.small_scene(6, 5, 4)
    sim = sph.Simulation(sc, params=dict(sc.params, max_neighbors=4, auto_rebuild=1))
    with pytest.raises(sph.SphError) as e:
        sim.step()
    assert e.value.code == sph.SPH_ERR_CAPACITY
    sim.close()


def test_free_fall_closed_form(sph):
    sc = scenes.small_scene(1, 1, 1, jitter=0.0, cfl_lambda=0.0, dt_max=1e-3)
    sc.x_fluid[:] = [[0.15, 0.2, 0.15]]
    sc.v_fluid[:] = [[0.3, 0.1, -0.2]]
    sim = sph.Simulation(sc)
    x0 = sc.x_fluid[0].astype(np.float64)
    v0 = sc.v_fluid[0].astype(np.float64)
    dt = float(np.float32(1e-3))
    g = np.array(sc.params["gravity"])
    for n in range(1, 21):
        st = sim.advance()
        assert st["iters_div"] == 0 and st["iters_dens"] == 0
    x = sim.read(("x",))["x"][0]
    expect = x0 + 20 * dt * v0 + g * dt * dt * 20 * 21 / 2
    np.testing.assert_allclose(x, expect, rtol=0, atol=2e-6)


def test_error_paths(sph):
    sc = scenes.small_scene(6, 5, 4)
    sim = sph.Simulation(sc)
    with pytest.raises(sph.SphError) as e:
        sim.step()                                  # no neighbours yet
    assert e.value.code == sph.SPH_ERR_STATE
    sim.close()
    tight = dict(sc.params, max_neighbors=4)
    sim = sph.Simulation(sc, params=tight)
    with pytest.raises(sph.SphError) as e:
        sim.build_neighbors()
    assert e.value.code == sph.SPH_ERR_CAPACITY
    sim.close()
    # empty fluid: the step runs and does nothing
    sc0 = scenes.small_scene(1, 1, 1)
    sc0.x_fluid = sc0.x_fluid[:0].copy()
    sc0.v_fluid = sc0.v_fluid[:0].copy()
    sim = sph.Simulation(sc0)
    st = sim.advance()
    assert st["iters_div"] == 0 and st["iters_dens"] == 0
    sim.close()


def test_implicit_viscosity_solution_property(sph):
    # zero warm start and no pressure iterations: the step's v is the CG solution
    sc = scenes.small_scene(8, 6, 6, visc_model=scenes.VISC_IMPLICIT, visc=10.0, warm_start=0,
                            cfl_lambda=0.0, dt_max=1e-3)
    sc.v_fluid[:] = np.random.default_rng(5).normal(0, 0.2, sc.v_fluid.shape).astype(np.float32)
    sim = sph.Simulation(sc)
    sim.set_forced_iters(0, 0)
    sim.build_neighbors()
    st = sim.step()
    g = sim.read(("v", "rho"))
    dt = st["dt"]
    b = sc.v_fluid.astype(np.float64) + dt * np.array(sc.params["gravity"])
    res = O.visc_residual(sc.params, sc.x_fluid, g["rho"].astype(np.float64), dt, b, g["v"].astype(np.float64))
    print("cg iters", st["cg_iters"], "gpu resid", st["cg_resid"], "oracle resid", res, flush=True)
    assert st["cg_iters"] > 0
    assert res <= 2 * sc.params["cg_tol"]
    x_ref, it, _ = O.visc_solve(sc.params, sc.x_fluid, dt, b)
    M, _ = O.visc_dense(sc.params, sc.x_fluid, dt)
    cond = np.linalg.cond(M)
    err = np.linalg.norm(g["v"].astype(np.float64).ravel() - x_ref.ravel()) / np.linalg.norm(x_ref)
    assert err <= 4 * cond * sc.params["cg_tol"]


def test_implicit_viscosity_cg_start_value(sph):
    # the CG start x0 = v~ + cg_warm_factor (v* - v~ of the previous step):
    # every step's v is still the solution (pressure off), the carried
    # correction is v* - v~ of the device's own step, the oracle run from the
    # re-anchored state (correction included) needs about as many iterations,
    # and the start saves iterations against x0 = v~ on the same scene
    def run(factor, steps=10):
        sc = scenes.small_scene(8, 10, 6, visc_model=scenes.VISC_IMPLICIT, visc=10.0, warm_start=0,
                                cfl_lambda=0.0, dt_max=1e-3, cg_warm_factor=factor)
        sc.v_fluid[:] = np.random.default_rng(7).normal(0, 0.2, sc.v_fluid.shape).astype(np.float32)
        sim = sph.Simulation(sc)
        sim.set_forced_iters(0, 0)
        local = O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid)
        total = 0
        for k in range(steps):
            sim.build_neighbors()
            state = oracle_state_from_gpu(sim, sc, local)
            st = sim.step()
            g = sim.read(("v", "rho", "dvisc"))
            dt = st["dt"]
            b = state.v.astype(np.float64) + dt * np.array(sc.params["gravity"])
            res = O.visc_residual(sc.params, state.x, g["rho"].astype(np.float64), dt, b, g["v"].astype(np.float64))
            assert res <= 2 * sc.params["cg_tol"], (factor, k, res)
            assert np.abs(g["dvisc"] - (g["v"] - b)).max() <= 1e-6 * (np.abs(b).max() + 1.0)
            if factor > 0 and k in (1, 5, 9):
                ref = O.step(state, forced_div=0, forced_dens=0)
                print("[cg start] step", k, "gpu", st["cg_iters"], "oracle", ref["cg_iters"], flush=True)
                assert abs(st["cg_iters"] - ref["cg_iters"]) <= 2 + ref["cg_iters"] // 5
            if k > 0:
                total += st["cg_iters"]
        sim.close()
        return total

    warm = run(0.5)
    cold = run(0.0)
    print("[cg start] iterations over 9 steps: start 0.5", warm, "x0 = v~", cold, flush=True)
    assert warm < cold


def test_c1_hundred_steps_statistics(sph):
    """Whole-run comparison on c1 (SPH is chaotic, so pointwise parity over
    many steps is unpinned): the GPU run and the oracle's own run from the
    same input, 100 steps each, every step within eta, iteration counts
    within one of each other step by step, and the fluid's centre of mass and
    front (largest x) within 1% at steps 10, 50 and 100, its kinetic energy
    within 1% at steps 10 and 50 and 2% at step 100.  The energy drifts
    fastest: with the bound on the largest compression a solve's stop can
    hang on one particle's predicted density, where the GPU's FP32 and the
    oracle's FP64 differ within rounding, so the two runs take a different
    iteration more often than with the mean alone (measured at step 100:
    1.4%, against 6e-4 before the bound)."""
    sc = scenes.scene("c1")
    p = sc.params
    m = p["rho0"] * (2.0 * p["r"]) ** 3
    sim = sph.Simulation(sc)
    state = O.State(sc, O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid))

    def stats(x, v):
        x = np.asarray(x, np.float64)
        v = np.asarray(v, np.float64)
        return x.mean(axis=0), 0.5 * m * float((v * v).sum()), float(x[:, 0].max())

    for k in range(100):
        st = sim.advance()
        out = O.step(state)
        state = O.advance(state, out)
        for which, eta in (("div", p["eta_divergence"]), ("dens", p["eta_density"])):
            assert st["err_" + which] <= eta or st["iters_" + which] == p["max_iters"], (k, which)
            assert out["err_" + which] <= eta or out["iters_" + which] == p["max_iters"], (k, which)
            assert abs(st["iters_" + which] - out["iters_" + which]) <= 1, (k, which, st, out["iters_" + which])
        if k in (9, 49, 99):
            g = sim.read(("x", "v"))
            cg, kg, fg = stats(g["x"], g["v"])
            cr, kr, fr = stats(state.x, state.v)
            print(f"step {k + 1}: com {cg} vs {cr}, ke {kg:.4f} vs {kr:.4f}, front {fg:.5f} vs {fr:.5f}", flush=True)
            assert np.all(np.abs(cg - cr) <= 0.01 * np.abs(cr)), (k, cg, cr)
            assert abs(kg - kr) <= (0.02 if k == 99 else 0.01) * kr, (k, kg, kr)
            assert abs(fg - fr) <= 0.01 * fr, (k, fg, fr)
            assert np.all(np.isfinite(g["x"])) and len(g["x"]) == sc.n_fluid
    sim.close()


@pytest.mark.parametrize("max_iters", [0, 1])
def test_iteration_cap(sph, max_iters):
    """The solves' cap (Alg. 2 with a limit): with no iteration allowed the
    step still integrates once with the warm start's pressure only; with one,
    every solve stops at one.  Both against the oracle run with the same cap."""
    sc = scenes.scene("c1")
    params = dict(sc.params, max_iters=max_iters)
    sim = sph.Simulation(sc, params=params)
    local = O.rigid_local(sc.x_boundary, sc.body_of_boundary, sc.rigid)
    worst = {}
    for k in range(3):
        sim.build_neighbors()
        state = oracle_state_from_gpu(sim, sc, local)
        st = sim.step()
        assert st["iters_div"] <= max_iters and st["iters_dens"] <= max_iters
        g = sim.read()
        for which in ("div", "dens"):
            eta = params["eta_divergence" if which == "div" else "eta_density"]
            assert st["iters_" + which] == max_iters or st["err_" + which] <= eta, (k, which, st)
        ref = O.step(state, forced_div=st["iters_div"], forced_dens=st["iters_dens"],
                     params=dict(state.params, max_iters=max_iters))
        r = compare_step(g, ref, st)
        for f, v in r.items():
            worst[f] = max(worst.get(f, 0.0), v)
    print("cap", max_iters, worst, flush=True)
    for f, v in worst.items():
        assert v <= 1.0, (f, v)
    sim.close()
