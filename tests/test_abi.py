"""The C ABI library loads without a GPU and exports every symbol its header declares."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(sph_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_header_declares_the_four_entry_points():
    names = declared_symbols()
    for n in ("sph_create", "sph_build_neighbors", "sph_step", "sph_read_state"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2403_11156_amd", "libsph.so")
    if not os.path.exists(lib_path):
        import __graft_entry__
        __graft_entry__.build()
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in sorted(declared_symbols()) if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_without_device():
    from paper_2403_11156_amd import sph
    assert sph.sph_strerror(0) == b"ok"
    assert sph.sph_strerror(-4) == b"neighbour capacity exceeded"


def test_create_rejects_invalid_arguments_without_device():
    # validation happens before any device call, so this runs on the CPU
    import numpy as np
    from paper_2403_11156_amd import scenes, sph
    sc = scenes.small_scene(2, 2, 2)
    bad = dict(sc.params, r=-1.0)
    try:
        sph.Simulation(sc, params=bad)
        raise AssertionError("accepted a negative radius")
    except sph.SphError as e:
        assert e.code == sph.SPH_ERR_INVALID
    sc.x_fluid[0, 0] = np.nan
    try:
        sph.Simulation(sc)
        raise AssertionError("accepted a NaN position")
    except sph.SphError as e:
        assert e.code == sph.SPH_ERR_INVALID


def test_create_rejects_bad_solver_settings_without_device():
    from paper_2403_11156_amd import scenes, sph
    sc = scenes.small_scene(2, 2, 2)
    for bad in (dict(sc.params, solver=3), dict(sc.params, solver=-1),
                dict(sc.params, solver=scenes.SOLVER_WCSPH, wcsph_k=0.0),
                dict(sc.params, solver=scenes.SOLVER_PCISPH, warm_start=scenes.WARM_LEARNED),
                dict(sc.params, solver=scenes.SOLVER_WCSPH, warm_start=scenes.WARM_LEARNED),
                dict(sc.params, separate_div_check=2), dict(sc.params, separate_div_check=-1),
                dict(sc.params, cg_warm_factor=5.0)):
        try:
            sph.Simulation(sc, params=bad)
            raise AssertionError(f"accepted {bad}")
        except sph.SphError as e:
            assert e.code == sph.SPH_ERR_INVALID


def test_required_bytes_without_device():
    # the arena size is computed by the allocation sequence of sph_create in
    # counting mode, without touching a device or the scene's arrays
    from paper_2403_11156_amd import scenes, sph
    small = scenes.small_scene(4, 4, 4)
    large = scenes.small_scene(8, 8, 8)
    a, b = sph.required_bytes(small), sph.required_bytes(large)
    assert a > 0 and b > a and a % 256 == 0 and b % 256 == 0
    # the implicit viscosity's CG vectors come on top
    c = sph.required_bytes(large, dict(large.params, visc_model=scenes.VISC_IMPLICIT, visc=1.0))
    assert c > b
    # per fluid particle at least the state, the lists and the solver fields
    per = (b - a) / (large.n_fluid - small.n_fluid)
    assert per > 4 * large.params["max_neighbors"]
    try:
        sph.required_bytes(small, dict(small.params, r=-1.0))
        raise AssertionError("accepted a negative radius")
    except sph.SphError as e:
        assert e.code == sph.SPH_ERR_INVALID


def test_misaligned_arena_is_rejected_before_any_device_call():
    # the arena's pieces are 256-byte aligned only if the arena is; a lent
    # pointer that is not is refused by the validation that precedes every
    # device call (the fake address below is never dereferenced; the case is
    # left to machines without a GPU all the same)
    import ctypes as C
    import numpy as np
    import pytest
    import torch
    from paper_2403_11156_amd import scenes, sph
    if torch.cuda.device_count() > 0:
        pytest.skip("uses a fake device address; run where no GPU is visible")
    s = scenes.small_scene(4, 4, 4)
    keep = [np.ascontiguousarray(s.x_fluid, np.float32), np.ascontiguousarray(s.v_fluid, np.float32),
            np.ascontiguousarray(s.x_boundary, np.float32).reshape(-1, 3),
            np.ascontiguousarray(s.body_of_boundary, np.int32)]
    sc = sph.sph_scene()
    sc.n_fluid, sc.n_boundary, sc.n_rigid = s.n_fluid, s.n_boundary, 0
    sc.x_fluid, sc.v_fluid, sc.x_boundary, sc.body_of_boundary = (sph._ptr(a) for a in keep)
    need = sph.required_bytes(s)
    sc.device_arena = C.c_void_p(0x7f0000000010)   # 16-byte, not 256-byte, aligned
    sc.device_arena_bytes = need + 4096
    p = sph.make_params(dict(s.params))
    ctx = C.c_void_p()
    rc = sph.sph_create(C.byref(p), C.byref(sc), None, C.byref(ctx))
    assert rc == sph.SPH_ERR_INVALID and not ctx.value
    assert b"256-byte aligned" in sph.sph_last_error(None)
