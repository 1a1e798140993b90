"""Seeded synthetic scenes for the DFSPH time step.

This module only places particles and rigid bodies; it holds none of the
method's arithmetic.  Both the HIP library (through the binding) and the CPU
oracle used by the tests consume exactly the arrays produced here.

Construction (a reading of the paper's scene set-up, Sec. 4.1 and Sec. 5):
  * y is up, gravity is (0, -9.81, 0).
  * The tank is a closed box whose interior is [lo, hi]; its walls are one
    layer of boundary particles (Akinci sampling, Sec. 3.5) on the planes
    lo - 1.2r and hi + 1.2r with a spacing within 1% of s = 2r.  A single
    Akinci layer at distance s from a fluid lattice plane over-covers that
    plane (rho = 1.064 rho0 on a face, 1.15 rho0 in a corner); at 1.1 s the
    wall-adjacent density starts within 0.5% of rho0.
  * Fluid sits on the cell-centred lattice r + s*i and every component is
    jittered by (2u - 1) * 0.1 r, u from SplitMix64(seed), computed in FP64
    and rounded to FP32 once.
  * Rigid bodies are boxes (surface points of a lattice of spacing s) and
    spheres (Fibonacci surface points at about one point per s^2).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

VISC_NONE, VISC_XSPH, VISC_LAPLACIAN, VISC_IMPLICIT = 0, 1, 2, 3
WARM_ZERO, WARM_PREVIOUS, WARM_LEARNED = 0, 1, 2
SOLVER_DFSPH, SOLVER_WCSPH, SOLVER_PCISPH = 0, 1, 2


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """The k-th output (k = offset .. offset+count-1) of SplitMix64 seeded
    with ``seed`` (Steele, Lea and Flood 2014): state_k = seed + (k+1)*gamma,
    then the variant-13 finaliser."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """u = (z >> 40) * 2^-24, a 24-bit uniform in [0, 1)."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def lattice(n, origin, spacing) -> np.ndarray:
    """Points origin + spacing * (i, j, k), x fastest, then y, then z (FP64)."""
    nx, ny, nz = n
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    k = np.arange(nz, dtype=np.float64)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    return np.asarray(origin, np.float64) + spacing * pts


def shell(n, origin, spacing) -> np.ndarray:
    """Surface points of an n[0] x n[1] x n[2] lattice (its outermost layer)."""
    nx, ny, nz = n
    pts = lattice(n, (0.0, 0.0, 0.0), 1.0)
    on = ((pts[:, 0] == 0) | (pts[:, 0] == nx - 1) | (pts[:, 1] == 0) |
          (pts[:, 1] == ny - 1) | (pts[:, 2] == 0) | (pts[:, 2] == nz - 1))
    return np.asarray(origin, np.float64) + spacing * pts[on]


WALL_OFFSET = 1.2  # wall planes sit WALL_OFFSET * r outside the interior


def tank_walls(lo, hi, r) -> np.ndarray:
    """One boundary layer on the planes lo - 1.2r and hi + 1.2r, i.e. 1.1 s
    from the outermost fluid lattice planes lo + r and hi - r, with the
    spacing closest to s that divides each span evenly."""
    s = 2.0 * r
    lo = np.asarray(lo, np.float64) - WALL_OFFSET * r
    hi = np.asarray(hi, np.float64) + WALL_OFFSET * r
    n = [int(round((hi[a] - lo[a]) / s)) + 1 for a in range(3)]
    pts = shell(n, (0.0, 0.0, 0.0), 1.0)
    step = np.array([(hi[a] - lo[a]) / (n[a] - 1) for a in range(3)])
    return lo + pts * step


def fibonacci_sphere(radius: float, spacing: float) -> np.ndarray:
    """About one point per spacing^2 on a sphere (golden-angle spiral)."""
    n = int(round(4.0 * math.pi * radius * radius / (spacing * spacing)))
    i = np.arange(n, dtype=np.float64)
    y = 1.0 - 2.0 * (i + 0.5) / n
    rad = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([np.cos(phi) * rad, y, np.sin(phi) * rad], axis=1)


def quat_to_matrix(q) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


@dataclasses.dataclass
class Scene:
    """One synthetic workload: parameters plus FP32 particle arrays."""
    name: str
    params: Dict
    x_fluid: np.ndarray            # (N_f, 3) float32
    v_fluid: np.ndarray            # (N_f, 3) float32
    x_boundary: np.ndarray         # (N_b, 3) float32
    body_of_boundary: np.ndarray   # (N_b,) int32, -1 = static tank
    rigid: List[Dict]              # mass, inertia(3), com(3), quat(4), vel(3), omega(3)
    steps: int
    seed: int

    @property
    def n_fluid(self) -> int:
        return int(self.x_fluid.shape[0])

    @property
    def n_boundary(self) -> int:
        return int(self.x_boundary.shape[0])


def default_params(r: float, lo, hi, **kw) -> Dict:
    p = dict(
        r=r, h=4.0 * r, rho0=1000.0, gravity=(0.0, -9.81, 0.0),
        domain_min=tuple(float(v) for v in lo), domain_max=tuple(float(v) for v in hi),
        eta_density=1e-3, eta_divergence=1e-3, max_iters=100,
        dt_max=1e-3, cfl_lambda=0.4,
        visc_model=VISC_XSPH, visc=0.01,
        cg_tol=1e-4, cg_max_iters=1000,
        # both solves start from 0.6 of the previous step's stiffness: with the
        # factor cap and the bound on the largest compression every configured
        # run stays bounded up to 0.65 (0.8 breaks down), and 0.6 needs fewer
        # iterations than 0.5 where the falling block is compressed
        warm_start=WARM_PREVIOUS, warm_factor=0.6,
        max_neighbors=64, max_boundary_neighbors=48,
        # WCSPH: gamma = 7, k = rho0 c^2 / gamma with a sound speed c of 44 m/s,
        # ten times the ~4.4 m/s a 1 m dam break reaches
        solver=SOLVER_DFSPH, wcsph_k=2.8e5, wcsph_gamma=7.0,
        # implicit viscosity: start the CG from v~ + 0.5 (v* - v~) of the previous step
        cg_warm_factor=0.5,
        # the DFSPH factor at most ten times its bulk-lattice value, and the
        # density solve also bounds the largest compression at 2%: without
        # them the dam breaks at 125k to 1.23M particles break down within
        # their configured lengths (a pair meeting at the support's edge, and
        # pockets of compression the mean error over a million particles hides)
        alpha_max_factor=10.0, eta_density_max=0.02,
        # bodies meet each other and the tank through frictionless contact
        # of their sample points, not the push-back into the tank
        rigid_contact=1,
    )
    p.update(kw)
    return p


def jittered_block(n, origin, r, seed, offset=0, jitter=0.1) -> np.ndarray:
    base = lattice(n, origin, 2.0 * r)
    u = uniform01(seed, base.size, offset).reshape(base.shape)
    return (base + (2.0 * u - 1.0) * jitter * r).astype(np.float32)


def make_block_scene(name, r, lo, hi, n_fluid, fluid_origin, seed, steps,
                     bodies: Optional[List[Dict]] = None, jitter: float = 0.1, **kw) -> Scene:
    params = default_params(r, lo, hi, **kw)
    xf = jittered_block(n_fluid, fluid_origin, r, seed, jitter=jitter)
    walls = tank_walls(lo, hi, r)
    xb = [walls]
    body = [np.full(len(walls), -1, np.int32)]
    rigid = []
    for bi, b in enumerate(bodies or []):
        pts = b["local_points"]
        R = quat_to_matrix(b["quat"])
        world = pts @ R.T + np.asarray(b["com"], np.float64)
        xb.append(world)
        body.append(np.full(len(world), bi, np.int32))
        rigid.append(dict(mass=b["mass"], inertia=tuple(b["inertia"]), com=tuple(b["com"]),
                          quat=tuple(b["quat"]), vel=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0)))
    return Scene(name=name, params=params, x_fluid=xf,
                 v_fluid=np.zeros_like(xf),
                 x_boundary=np.concatenate(xb).astype(np.float32),
                 body_of_boundary=np.concatenate(body).astype(np.int32),
                 rigid=rigid, steps=steps, seed=seed)


def _random_yaw_quat(u) -> tuple:
    ang = 2.0 * math.pi * u
    return (math.cos(ang / 2), 0.0, math.sin(ang / 2), 0.0)


def _random_quat(u1, u2, u3) -> tuple:
    # Shoemake's uniform random rotation.
    a = math.sqrt(1 - u1)
    b = math.sqrt(u1)
    return (b * math.cos(2 * math.pi * u3), a * math.sin(2 * math.pi * u2),
            a * math.cos(2 * math.pi * u2), b * math.sin(2 * math.pi * u3))


def rigid_bodies_c3(r: float, seed: int, centres=None) -> List[Dict]:
    """Two boxes (0.2 m, 500 and 600 kg/m^3) and two spheres (R 0.15 m,
    700 and 800 kg/m^3) at x = 1.75 (or at the four given centres),
    centres jittered by +-0.01 m."""
    s = 2.0 * r
    u = uniform01(seed, 16, offset=10_000_000)
    out = []
    if centres is None:
        centres = [(1.75, 0.5, 0.25), (1.75, 0.5, 0.75), (1.75, 0.8, 0.25), (1.75, 0.8, 0.75)]
    specs = [("box", 0.2, 500.0, centres[0]), ("box", 0.2, 600.0, centres[1]),
             ("sphere", 0.15, 700.0, centres[2]), ("sphere", 0.15, 800.0, centres[3])]
    for bi, (kind, size, dens, c) in enumerate(specs):
        com = tuple(c[a] + (2.0 * u[4 * bi + a] - 1.0) * 0.01 for a in range(3))
        if kind == "box":
            n = int(round(size / s)) + 1
            pts = shell((n, n, n), (-size / 2,) * 3, s)
            mass = dens * size ** 3
            inertia = (mass * size * size / 6.0,) * 3
            # yaw only, so the boxes keep their vertical extent and never
            # overlap the spheres stacked above them
            quat = _random_yaw_quat(u[4 * bi + 3])
        else:
            pts = fibonacci_sphere(size, s)
            mass = dens * 4.0 / 3.0 * math.pi * size ** 3
            inertia = (0.4 * mass * size * size,) * 3
            uu = uniform01(seed, 3, offset=20_000_000 + 3 * bi)
            quat = _random_quat(*uu)
        out.append(dict(local_points=pts, mass=mass, inertia=inertia, com=com, quat=quat, kind=kind, size=size))
    return out


def carve(x: np.ndarray, bodies: List[Dict], gap: float) -> np.ndarray:
    """The fluid points that lie at least `gap` outside every body (boxes:
    in the body frame, |q_a| >= size/2 + gap on some axis; spheres:
    distance >= R + gap from the centre)."""
    keep = np.ones(len(x), bool)
    for b in bodies:
        d = x.astype(np.float64) - np.asarray(b["com"], np.float64)
        if b["kind"] == "box":
            q = d @ quat_to_matrix(b["quat"])   # R^T d, row-wise
            keep &= (np.abs(q) >= 0.5 * b["size"] + gap).any(axis=1)
        else:
            keep &= np.linalg.norm(d, axis=1) >= b["size"] + gap
    return x[keep]


def scene(name: str) -> Scene:
    """Named workloads.  c1..c5 are the benchmark scenes; the others are
    small physics fixtures."""
    name = name.lower()
    if name == "c1":
        # 20^3 = 8000 fluid in a 0.8 m cube, fixed dt 4e-4, XSPH 0.01
        return make_block_scene("c1 dam break 8k", 0.01, (0, 0, 0), (0.8, 0.8, 0.8), (20, 20, 20),
                                (0.01, 0.01, 0.01), seed=1, steps=100, cfl_lambda=0.0, dt_max=4e-4)
    if name == "c2":
        return make_block_scene("c2 dam break 125k", 0.01, (0, 0, 0), (2.0, 1.0, 1.0), (50, 50, 50),
                                (0.01, 0.01, 0.01), seed=2, steps=1000)
    if name == "c3":
        return make_block_scene("c3 rigid coupling 1.23M", 0.005, (0, 0, 0), (2.0, 1.0, 1.0),
                                (150, 82, 100), (0.005, 0.175, 0.005), seed=3, steps=500,
                                bodies=rigid_bodies_c3(0.005, 3))
    if name == "c3i":
        # c3 with the four bodies inside the block (boxes low, spheres above
        # them), the fluid carved away within 1.1 s of their surfaces, as the
        # tank walls stand 1.1 s from the fluid: the coupling under load
        r = 0.005
        bodies = rigid_bodies_c3(r, 3, centres=[(0.45, 0.45, 0.3), (0.45, 0.45, 0.7), (1.05, 0.6, 0.3),
                                                (1.05, 0.6, 0.7)])
        sc = make_block_scene("c3 rigid coupling 1.23M, bodies immersed", r, (0, 0, 0), (2.0, 1.0, 1.0),
                              (150, 82, 100), (0.005, 0.175, 0.005), seed=3, steps=500, bodies=bodies)
        sc.x_fluid = np.ascontiguousarray(carve(sc.x_fluid, bodies, 2.2 * r))
        sc.v_fluid = np.zeros_like(sc.x_fluid)
        return sc
    if name == "c4":
        return make_block_scene("c4 viscous column 250k", 0.008, (0, 0, 0), (3.2, 2.0, 0.8),
                                (50, 100, 50), (0.008, 0.008, 0.008), seed=4, steps=500,
                                visc_model=VISC_IMPLICIT, visc=10.0)
    if name == "c5":
        return make_block_scene("c5 dam break 1.23M", 0.005, (0, 0, 0), (2.0, 1.0, 1.0),
                                (150, 82, 100), (0.005, 0.005, 0.005), seed=5, steps=1000)
    if name == "c1w":
        # c1 with the WCSPH solver; dt within the acoustic limit 0.4 h / c
        return make_block_scene("c1 dam break 8k, WCSPH", 0.01, (0, 0, 0), (0.8, 0.8, 0.8), (20, 20, 20),
                                (0.01, 0.01, 0.01), seed=1, steps=100, cfl_lambda=0.0, dt_max=2e-4,
                                solver=SOLVER_WCSPH)
    if name == "c5w":
        return make_block_scene("c5 dam break 1.23M, WCSPH", 0.005, (0, 0, 0), (2.0, 1.0, 1.0),
                                (150, 82, 100), (0.005, 0.005, 0.005), seed=5, steps=1000, dt_max=1.5e-4,
                                solver=SOLVER_WCSPH)
    if name == "c1p":
        # c1 with the PCISPH solver (density solve only, pressure from zero each step)
        return make_block_scene("c1 dam break 8k, PCISPH", 0.01, (0, 0, 0), (0.8, 0.8, 0.8), (20, 20, 20),
                                (0.01, 0.01, 0.01), seed=1, steps=100, cfl_lambda=0.0, dt_max=4e-4,
                                solver=SOLVER_PCISPH, warm_start=WARM_ZERO)
    if name == "c5p":
        return make_block_scene("c5 dam break 1.23M, PCISPH", 0.005, (0, 0, 0), (2.0, 1.0, 1.0),
                                (150, 82, 100), (0.005, 0.005, 0.005), seed=5, steps=1000,
                                solver=SOLVER_PCISPH, warm_start=WARM_ZERO)
    if name == "column":
        # hydrostatic fixture: unjittered 10 x 30 x 10 column filling a 0.2 m wide tank
        return make_block_scene("hydrostatic column", 0.01, (0, 0, 0), (0.2, 0.8, 0.2), (10, 30, 10),
                                (0.01, 0.01, 0.01), seed=7, steps=2500, jitter=0.0, cfl_lambda=0.0,
                                dt_max=4e-4)
    raise KeyError(name)


def small_scene(nx=6, ny=5, nz=4, r=0.01, seed=11, tank=(0.3, 0.3, 0.3), origin=None,
                bodies=None, **kw) -> Scene:
    """A small dam-break block for parity tests (a few hundred particles)."""
    if origin is None:
        origin = (r, r, r)
    return make_block_scene(f"small {nx}x{ny}x{nz}", r, (0, 0, 0), tank, (nx, ny, nz), origin,
                            seed=seed, steps=10, bodies=bodies, **kw)


def small_bodies(r: float, seed: int, centres) -> List[Dict]:
    """Small boxes (side 6s) for rigid-coupling parity tests."""
    s = 2.0 * r
    out = []
    u = uniform01(seed, 4 * len(centres), offset=30_000_000)
    for bi, c in enumerate(centres):
        size = 6 * s
        pts = shell((7, 7, 7), (-size / 2,) * 3, s)
        mass = 500.0 * size ** 3
        out.append(dict(local_points=pts, mass=mass, inertia=(mass * size * size / 6.0,) * 3,
                        com=tuple(c), quat=_random_quat(u[4 * bi], u[4 * bi + 1], u[4 * bi + 2]), kind="box",
                        size=size))
    return out
