"""The device's pressure pass on the exact lattice of the oracle's operator
pins (r = 2^-7, h = 2s, a 9^3 block far from any wall): a stiffness that
alternates between y layers moves no bulk particle (the odd-even null space
of Eq. 7 on the lattice), and a stiffness falling linearly with height
pushes every bulk particle up by the closed form, dt m |b| (k/h) sum_j
|f'(q_j)| dy_j^2 / r_j for kappa/rho = c0 + b y, i.e. a hydrostatic profile
K = g (H - y) balances gravity to the lattice factor F = 1.0201.  FP32 sums
on the device against FP64 closed forms."""

import math

import numpy as np
import pytest

from paper_2403_11156_amd import scenes

pytestmark = pytest.mark.gpu

R = 2.0 ** -7
S = 2.0 * R
H = 2.0 * S
RHO0 = 1000.0
M = RHO0 * S ** 3
KN = 8.0 / (math.pi * H ** 3)
Q1, Q2, Q3 = 0.5, 1.0 / math.sqrt(2.0), math.sqrt(3.0) / 2.0


def f(q):
    return 6.0 * (q ** 3 - q ** 2) + 1.0 if q <= 0.5 else 2.0 * (1.0 - q) ** 3


def fp(q):
    return 6.0 * (3.0 * q * q - 2.0 * q) if q <= 0.5 else -6.0 * (1.0 - q) ** 2


RHO_LAT = RHO0 * (1.0 + 6 * f(Q1) + 12 * f(Q2) + 8 * f(Q3)) / math.pi
LAT = S * (2.0 * abs(fp(Q1)) + 8.0 * abs(fp(Q2)) / math.sqrt(2.0) + 8.0 * abs(fp(Q3)) / math.sqrt(3.0))
WF = 0.5


@pytest.fixture(scope="module")
def sph():
    import torch
    assert torch.cuda.is_available()
    from paper_2403_11156_amd import sph as mod
    return mod


def _lattice_scene():
    # the 9^3 block at the centre of a unit tank; a small static wall far
    # below it (no boundary neighbours); no gravity, viscosity, cap or bound
    x = scenes.lattice((9, 9, 9), (0.5 - 4 * S,) * 3, S).astype(np.float32)
    sc = scenes.make_block_scene("lattice", R, (0, 0, 0), (1, 1, 1), (1, 1, 1), (0.5, 0.5, 0.5), seed=1, steps=1,
                                 jitter=0.0, gravity=(0.0, 0.0, 0.0), visc_model=scenes.VISC_NONE,
                                 warm_start=scenes.WARM_PREVIOUS, warm_factor=WF, cfl_lambda=0.0, dt_max=1e-4,
                                 alpha_max_factor=0.0, eta_density_max=0.0)
    sc.x_fluid = x
    sc.v_fluid = np.zeros_like(x)
    sc.x_boundary = scenes.lattice((5, 1, 5), (0.5 - 2 * S, 0.1, 0.5 - 2 * S), S).astype(np.float32)
    sc.body_of_boundary = np.full(len(sc.x_boundary), -1, np.int32)
    sc.rigid = []
    idx3 = np.rint((x.astype(np.float64) - x.min(axis=0)) / S).astype(int)
    bulk = np.all((idx3 >= 2) & (idx3 <= 6), axis=1)   # whole neighbourhoods of bulk density
    assert bulk.sum() == 125
    return sc, idx3[:, 1], bulk


def _step_with_stiffness(sph, sc, K):
    sim = sph.Simulation(sc)
    sim.write(K=np.asarray(K, np.float32))   # the previous step's stiffness, which the warm start scales
    sim.build_neighbors()
    sim.set_forced_iters(0, 0)
    st = sim.step()
    g = sim.read(("v", "rho"))
    sim.close()
    return st, g


def test_layer_alternating_stiffness_moves_no_bulk_particle(sph):
    sc, layer, bulk = _lattice_scene()
    for K in (np.where(layer % 2 == 0, 64.0, 16.0), np.where(layer % 2 == 0, 0.0, 40.0)):
        st, g = _step_with_stiffness(sph, sc, K)
        np.testing.assert_allclose(g["rho"][bulk], RHO_LAT, rtol=1e-6)
        scale = st["dt"] * M * WF * K.max() / RHO_LAT * KN / H * 6.0 * 27
        worst = np.abs(g["v"][bulk]).max() / scale
        print(f"[lattice] alternating K {K.min():g}/{K.max():g}: bulk |v| / term scale {worst:.2e}", flush=True)
        assert worst < 1e-6


def test_linear_stiffness_pushes_the_bulk_by_the_closed_form(sph):
    sc, layer, bulk = _lattice_scene()
    st, g = _step_with_stiffness(sph, sc, 64.0 - 6.0 * layer)
    vy = g["v"][bulk, 1].astype(np.float64)
    F = M / RHO_LAT * KN / H * LAT
    expect = st["dt"] * (WF * 6.0 / S) * F
    print(f"[lattice] ramp: bulk v_y {vy.min():.7e}..{vy.max():.7e}, closed form {expect:.7e} (F = {F:.6f})",
          flush=True)
    np.testing.assert_allclose(vy, expect, rtol=2e-5, atol=0)
    assert np.abs(g["v"][bulk][:, [0, 2]]).max() < 1e-5 * expect
