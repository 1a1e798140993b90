"""State exchange through the C ABI: read-back after later sorts, checkpoint
and resume, and the non-finite-state error."""

import numpy as np
import pytest

from paper_2403_11156_amd import scenes

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "rho", "alpha", "K", "Kv", "kappa", "accel", "nbr")


@pytest.fixture(scope="module")
def sph():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_11156_amd import sph as mod
    return mod


def _bodies_scene():
    r = 0.01
    bodies = scenes.small_bodies(r, 4, [(0.22, 0.12, 0.2)])
    return scenes.make_block_scene("small+body", r, (0, 0, 0), (0.4, 0.3, 0.4), (9, 7, 8), (0.012, 0.012, 0.012),
                                   seed=6, steps=4, bodies=bodies)


def _same(a, b, where):
    for f in a:
        assert np.array_equal(a[f], b[f]), (where, f)


def test_read_back_after_later_sorts(sph):
    # a step's alpha, kappa, acceleration and neighbour counts stay in the
    # order of the step that wrote them; read back after one and after two
    # later sorts (explicit builds) they must still land on their particles
    sc = scenes.scene("c1")
    sim = sph.Simulation(sc)
    for _ in range(3):
        sim.build_neighbors()
        sim.step()
    ref = sim.read(FIELDS)
    sim.build_neighbors()
    _same(ref, sim.read(FIELDS), "one build")
    sim.build_neighbors()
    _same(ref, sim.read(FIELDS), "two builds")
    sim.close()
    # auto_rebuild: the step queues the next sort itself; a write of the same
    # state and an explicit build follow
    sim = sph.Simulation(sc, params=dict(sc.params, auto_rebuild=1))
    for _ in range(3):
        sim.advance()
    ref = sim.read(FIELDS)
    sim.write(x=ref["x"], v=ref["v"])
    _same(ref, sim.read(FIELDS), "write after a queued build")
    sim.build_neighbors()
    _same(ref, sim.read(FIELDS), "build after a queued build")
    sim.close()


@pytest.mark.parametrize("name", ["c1", "bodies"])
def test_checkpoint_resume_is_bit_identical(sph, name):
    # a fresh context given the state read from a running one (x, v, rho, K,
    # Kv, boundary, rigid) continues it bit for bit
    sc = scenes.scene("c1") if name == "c1" else _bodies_scene()
    params = dict(sc.params, auto_rebuild=1, separate_div_check=1)
    a = sph.Simulation(sc, params=params)
    for _ in range(5):
        a.advance()
    ck = a.read(("x", "v", "rho", "K", "Kv", "boundary", "rigid"))
    b = sph.Simulation(sc, params=params)
    b.write(x=ck["x"], v=ck["v"], rho=ck["rho"], K=ck["K"], Kv=ck["Kv"], xb=ck["xb"], vb=ck["vb"],
            rigid=ck.get("rigid"))
    for k in range(4):
        sa, sb = a.advance(), b.advance()
        for key in ("dt", "iters_div", "iters_dens", "err_div", "err_dens", "nbr_min", "nbr_max"):
            assert sa[key] == sb[key], (k, key, sa[key], sb[key])
        ra = a.read(FIELDS + ("boundary", "rigid"))
        rb = b.read(FIELDS + ("boundary", "rigid"))
        for f in ra:
            if f == "rigid":
                for ba, bb in zip(ra[f], rb[f]):
                    for key in ba:
                        assert np.array_equal(np.asarray(ba[key]), np.asarray(bb[key])), (k, key)
            else:
                assert np.array_equal(ra[f], rb[f]), (k, f)
    # without the density the divergence warm start differs at once
    c = sph.Simulation(sc, params=params)
    c.write(x=ck["x"], v=ck["v"], K=ck["K"], Kv=ck["Kv"], xb=ck["xb"], vb=ck["vb"], rigid=ck.get("rigid"))
    d = sph.Simulation(sc, params=params)
    d.write(x=ck["x"], v=ck["v"], rho=ck["rho"], K=ck["K"], Kv=ck["Kv"], xb=ck["xb"], vb=ck["vb"],
            rigid=ck.get("rigid"))
    c.advance()
    d.advance()
    assert not np.array_equal(c.read(("v",))["v"], d.read(("v",))["v"])
    for s in (a, b, c, d):
        s.close()


def test_non_finite_state_is_reported(sph):
    # a NaN velocity (written from the host) reaches the solver's error, which
    # the step reports as SPH_ERR_NUMERIC instead of a converged step; every
    # kernel runs to its end on the NaN arithmetic
    sc = scenes.scene("c1")
    sim = sph.Simulation(sc)
    sim.build_neighbors()
    sim.step()
    v = sim.read(("v",))["v"]
    v[123] = np.nan
    sim.write(v=v)
    sim.build_neighbors()
    with pytest.raises(sph.SphError) as e:
        sim.step()
    assert e.value.code == sph.SPH_ERR_NUMERIC
    sim.close()


def test_write_rejects_a_non_positive_density(sph):
    sc = scenes.small_scene(3, 3, 3)
    sim = sph.Simulation(sc)
    rho = np.full(sc.n_fluid, 1000.0, np.float32)
    rho[2] = 0.0
    with pytest.raises(sph.SphError) as e:
        sim.write(rho=rho)
    assert e.value.code == sph.SPH_ERR_INVALID
    sim.close()


@pytest.mark.parametrize("name", ["c1", "bodies", "implicit"])
def test_borrowed_arena_runs_bit_identical(sph, name):
    # every device buffer carved from a torch-owned tensor: the same bits as
    # the context's own allocations over five steps; the arena is not freed
    # by the library and a one-byte-short arena is refused before any use
    import torch
    if name == "c1":
        sc = scenes.scene("c1")
    elif name == "bodies":
        sc = _bodies_scene()
    else:
        sc = scenes.small_scene(8, 6, 6, visc_model=scenes.VISC_IMPLICIT, visc=10.0)
    pd = dict(sc.params, auto_rebuild=1)
    need = sph.required_bytes(sc, pd)
    print(f"[arena] {name}: {need} bytes for {sc.n_fluid} fluid, {sc.n_boundary} boundary", flush=True)
    ref = sph.Simulation(sc, params=pd)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    sim = sph.Simulation(sc, params=pd, arena=arena)
    assert sim.info()["device_bytes"] == need
    for _ in range(5):
        a, b = ref.advance(), sim.advance()
        assert a["iters_dens"] == b["iters_dens"] and a["dt"] == b["dt"]
    fields = FIELDS + (("rigid",) if sc.rigid else ())
    ga, gb = ref.read(fields), sim.read(fields)
    for f in ga:
        if f == "rigid":
            assert ga[f] == gb[f]
        else:
            assert np.array_equal(ga[f], gb[f]), f
    sim.close()
    ref.close()
    arena.fill_(0)   # still the caller's memory
    torch.cuda.synchronize()
    short = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sph.SphError) as e:
        sph.Simulation(sc, params=pd, arena=short)
    assert e.value.code == sph.SPH_ERR_OOM
