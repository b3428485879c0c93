"""Seeded synthetic scenes for the batched MLS-MPM substep.

This module only draws inputs: particle positions, velocities and the scalar
settings of each environment. It holds none of the simulation arithmetic, so
both the HIP path and the FP64 oracle can be fed from it without sharing any
of the method.

Every array is drawn in float64 from ``numpy.random.Generator(PCG64(seed))``
and rounded to float32; the oracle receives the same float32 values upcast.

The workloads stand in for the paper's MPM task scenes (Appendix E tables for
RollingFlat, HandFlip and FluidMove: 48^3 grids, a few thousand particles,
dt = 5e-5, E of a few thousand, nu = 0.2, sigma_y 50-130), whose robot and
tool assets are not available. Sizes follow the five benchmark workloads:

* ``single_nh``      1 env, 32^3, 4,096 neo-Hookean particles, 10 substeps.
* ``batched_corot``  32 identical envs, 48^3, 20,000 corotated particles each.
* ``uneven_mixed``   64 envs, 64^3, 5k-60k particles of three materials.
* ``dam_break``      16 envs, 96^3, 200k Tait-fluid particles + moving gate.
* ``serving``        a Poisson stream of single-env rollout requests.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Material identifiers shared with the C header (interface constants).
NEOHOOKEAN = 0
COROTATED = 1
VONMISES = 2
FLUID_TAIT = 3
FLUID_PAPER = 4
MATERIAL_NAMES = {
    NEOHOOKEAN: "neohookean",
    COROTATED: "corotated",
    VONMISES: "vonmises",
    FLUID_TAIT: "fluid_tait",
    FLUID_PAPER: "fluid_paper",
}

GRAVITY = (0.0, 0.0, -9.8)  # z is up (Appendix E notation)
WALL = 3                    # sticky boundary thickness in nodes


@dataclass
class BoxCollider:
    """A kinematic box (or ball) moving at constant velocity and spinning at a
    constant rate about a fixed axis through its center (one-way coupling)."""
    center: tuple
    half: tuple
    velocity: tuple
    alpha: float      # softness of the contact blend, 1/length
    mu_b: float       # Coulomb friction coefficient
    axis: tuple = (0.0, 0.0, 1.0)   # rotation axis (unit)
    angle: float = 0.0              # rotation about the axis at t = 0 (rad)
    omega: float = 0.0              # angular speed (rad/s)
    shape: str = "box"              # "box", or "sphere": a ball of radius half[0]
    rounding: float = 0.0           # a box's distance less this radius (half (h, 0, 0): a capsule)

    @property
    def rotates(self) -> bool:
        return self.angle != 0.0 or self.omega != 0.0


def sphere_collider(center, radius: float, velocity, alpha: float, mu_b: float, **kw) -> BoxCollider:
    """A kinematic ball of the given radius (the collider with shape "sphere")."""
    r = float(radius)
    return BoxCollider(center=tuple(center), half=(r, r, r), velocity=tuple(velocity), alpha=alpha, mu_b=mu_b,
                       shape="sphere", **kw)


def capsule_collider(center, half_length: float, radius: float, velocity, alpha: float, mu_b: float,
                     **kw) -> BoxCollider:
    """A kinematic capsule: a segment of the given half length along the collider's own x axis, inflated by
    `radius` (the box of half extents (half_length, 0, 0) rounded by the radius)."""
    return BoxCollider(center=tuple(center), half=(float(half_length), 0.0, 0.0), velocity=tuple(velocity),
                       alpha=alpha, mu_b=mu_b, rounding=float(radius), **kw)


@dataclass
class EnvSpec:
    n: int                       # grid nodes per axis, domain [0,1]^3, dx = 1/n
    dt: float
    material: int
    E: float = 0.0
    nu: float = 0.0
    rho: float = 1e3
    Vp: float = 0.0              # particle volume
    sigma_y: float = 0.0
    K: float = 0.0               # Tait bulk modulus
    gamma: float = 0.0           # Tait exponent
    gravity: tuple = GRAVITY
    wall: int = WALL
    collider: Optional[BoxCollider] = None
    more_colliders: tuple = ()   # further colliders, applied after `collider` in order
    x: np.ndarray = None         # [N,3] float32
    v: np.ndarray = None         # [N,3] float32
    C: np.ndarray = None         # [N,3,3] float32
    F: np.ndarray = None         # [N,3,3] float32

    @property
    def n_particles(self) -> int:
        return 0 if self.x is None else int(self.x.shape[0])

    def params(self) -> np.ndarray:
        """The 8-entry parameter row of the C interface: E, nu, rho, Vp, sigma_y, K, gamma, 0."""
        return np.array([self.E, self.nu, self.rho, self.Vp, self.sigma_y,
                         self.K, self.gamma, 0.0], dtype=np.float64)

    def copy(self) -> "EnvSpec":
        out = dataclasses.replace(self)
        for k in ("x", "v", "C", "F"):
            a = getattr(self, k)
            setattr(out, k, None if a is None else a.copy())
        return out


@dataclass
class Workload:
    name: str
    envs: List[EnvSpec]
    substeps: int
    ckpt_every: int
    loss_weights: List[np.ndarray] = field(default_factory=list)  # per env [N,3] float32

    @property
    def n_particles(self) -> int:
        return sum(e.n_particles for e in self.envs)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _rest_state(N: int):
    C = np.zeros((N, 3, 3), dtype=np.float32)
    F = np.broadcast_to(np.eye(3, dtype=np.float32), (N, 3, 3)).copy()
    return C, F


def jittered_lattice(rng, lo: float, count: int, spacing: float) -> np.ndarray:
    """count^3 points at lo + (i + 1/2) h, each axis jittered by U(-h/4, h/4)."""
    i = np.arange(count, dtype=np.float64)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)
    pts = lo + (g + 0.5) * spacing + rng.uniform(-0.25 * spacing, 0.25 * spacing, size=g.shape)
    return _f32(pts)


def random_box(rng, lo_side=0.15, hi_side=0.3):
    side = rng.uniform(lo_side, hi_side, size=3)
    center = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    return center - side / 2, side


def uniform_points(rng, lo, side, N) -> np.ndarray:
    return _f32(lo + rng.uniform(0.0, 1.0, size=(N, 3)) * side)


def single_nh(seed: int = 0, weight_seed: int = 1, n_substeps: int = 10) -> Workload:
    """One neo-Hookean jelly cube: 16^3 jittered lattice inside [0.3, 0.5]^3 on 32^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    N = 16 ** 3
    x = jittered_lattice(rng, 0.3, 16, 0.2 / 16)
    v = _f32(rng.uniform(-0.5, 0.5, size=(N, 3)))
    C, F = _rest_state(N)
    env = EnvSpec(n=32, dt=1e-4, material=NEOHOOKEAN, E=5e3, nu=0.3, rho=1e3,
                  Vp=0.2 ** 3 / N, x=x, v=v, C=C, F=F)
    wr = np.random.Generator(np.random.PCG64(weight_seed))
    w = _f32(wr.standard_normal((N, 3)))
    return Workload("single_nh", [env], n_substeps, n_substeps, [w])


def batched_corot(seed: int = 2, n_envs: int = 32, n_per_env: int = 20000,
                  n_substeps: int = 80, ckpt_every: int = 10) -> Workload:
    """n_envs identical corotated boxes (random box drawn once) on 48^3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, side = random_box(rng)
    x = uniform_points(rng, lo, side, n_per_env)
    v = _f32(rng.uniform(-0.5, 0.5, size=(n_per_env, 3)))
    C, F = _rest_state(n_per_env)
    base = EnvSpec(n=48, dt=5e-5, material=COROTATED, E=1e4, nu=0.25, rho=1e3,
                   Vp=float(np.prod(side)) / n_per_env, x=x, v=v, C=C, F=F)
    w = _f32(rng.standard_normal((n_per_env, 3)))
    envs = [base.copy() for _ in range(n_envs)]
    return Workload("batched_corot", envs, n_substeps, ckpt_every, [w.copy() for _ in envs])


def handflip_shape(seed: int = 6, n_envs: int = 128, n_per_env: int = 2500, n_substeps: int = 40,
                   ckpt_every: int = 10) -> Workload:
    """The shape of the paper's own MPM throughput study (HandFlip: 48^3 grid,
    2,500 dough particles per env, von Mises E = 4000, nu = 0.2, sigma_y = 130,
    rho = 1, 40 substeps per frame, up to 128 envs). The hand is not modelled:
    each env is a seeded block of dough of side 0.14 moving at random
    velocities, which stands in for the hand-driven scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    envs, ws = [], []
    side = np.full(3, 0.14)
    for _ in range(n_envs):
        lo = 0.5 - side / 2 + rng.uniform(-0.05, 0.05, size=3)
        x = uniform_points(rng, lo, side, n_per_env)
        v = _f32(rng.uniform(-0.5, 0.5, size=(n_per_env, 3)))
        C, F = _rest_state(n_per_env)
        envs.append(EnvSpec(n=48, dt=5e-5, material=VONMISES, E=4000.0, nu=0.2, rho=1.0, sigma_y=130.0,
                            Vp=float(np.prod(side)) / n_per_env, x=x, v=v, C=C, F=F))
        ws.append(_f32(rng.standard_normal((n_per_env, 3))))
    return Workload("handflip_shape", envs, n_substeps, ckpt_every, ws)


def handflip_gripper(seed: int = 6, n_envs: int = 128, n_per_env: int = 2500, n_substeps: int = 40,
                     ckpt_every: int = 10) -> Workload:
    """handflip_shape with a four-finger gripper in every env: four capsules
    (half length 0.06, radius 0.02) around the dough block, closing in on it
    from four sides and turning slowly about their own axis, so the grid
    passes run their several-collider variant."""
    wl = handflip_shape(seed, n_envs, n_per_env, n_substeps, ckpt_every)
    envs = []
    for e in wl.envs:
        c = e.x.mean(0).astype(np.float64)
        fingers = []
        for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            ctr = (float(c[0] + 0.1 * dx), float(c[1] + 0.1 * dy), float(c[2]))
            fingers.append(capsule_collider(center=ctr, half_length=0.06, radius=0.02,
                                            velocity=(-0.3 * dx, -0.3 * dy, 0.0), alpha=96.0, mu_b=0.5,
                                            axis=(0.0, 0.0, 1.0), angle=0.5 * math.pi * abs(dy), omega=0.5))
        envs.append(dataclasses.replace(e, collider=fingers[0], more_colliders=tuple(fingers[1:])))
    return Workload("handflip_gripper", envs, n_substeps, ckpt_every, wl.loss_weights)


MIXED_MATERIALS = (
    dict(material=NEOHOOKEAN, E=5e3, nu=0.3),
    dict(material=VONMISES, E=5e3, nu=0.2, sigma_y=50.0),
    dict(material=FLUID_TAIT, K=1e4, gamma=7.0),
)


def uneven_mixed(seed: int = 3, n_envs: int = 64, n_lo: int = 5000, n_hi: int = 60000,
                 n_substeps: int = 50, ckpt_every: int = 10, grid: int = 64) -> Workload:
    """Envs of uneven size; material uniform over NH / von Mises / Tait fluid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    envs, ws = [], []
    for _ in range(n_envs):
        N = int(rng.integers(n_lo, n_hi + 1))
        mat = MIXED_MATERIALS[int(rng.integers(0, 3))]
        lo, side = random_box(rng)
        x = uniform_points(rng, lo, side, N)
        v = _f32(rng.uniform(-0.5, 0.5, size=(N, 3)))
        C, F = _rest_state(N)
        envs.append(EnvSpec(n=grid, dt=5e-5, rho=1e3, Vp=float(np.prod(side)) / N,
                            x=x, v=v, C=C, F=F, **mat))
        ws.append(_f32(rng.standard_normal((N, 3))))
    return Workload("uneven_mixed", envs, n_substeps, ckpt_every, ws)


def dam_break(seed: int = 4, n_envs: int = 16, n_per_env: int = 200000, grid: int = 96,
              n_substeps: int = 100, ckpt_every: int = 20) -> Workload:
    """Tait-fluid column (30% of the walled interior) held by a gate withdrawn at 0.2 m/s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = WALL / grid
    L = 1.0 - 2 * b
    lo = np.array([b, b, b])
    side = np.array([0.4 * L, L, 0.75 * L])          # 0.4 * 1 * 0.75 = 30% of L^3
    gate = BoxCollider(center=(b + 0.4 * L + 0.02, 0.5, b + 0.4 * L),
                       half=(0.02, 0.5 * L, 0.4 * L), velocity=(0.2, 0.0, 0.0),
                       alpha=2.0 * grid, mu_b=0.5)
    envs, ws = [], []
    # keep particles half a cell inside the walled box so the stencil band holds
    pad = 0.5 / grid
    for _ in range(n_envs):
        x = uniform_points(rng, lo + pad, side - 2 * pad, n_per_env)
        v = np.zeros((n_per_env, 3), dtype=np.float32)
        C, F = _rest_state(n_per_env)
        envs.append(EnvSpec(n=grid, dt=2e-5, material=FLUID_TAIT, K=1e4, gamma=7.0, rho=1e3,
                            Vp=float(np.prod(side)) / n_per_env, collider=gate,
                            x=x, v=v, C=C, F=F))
        ws.append(_f32(rng.standard_normal((n_per_env, 3))))
    return Workload("dam_break", envs, n_substeps, ckpt_every, ws)


@dataclass
class Request:
    rid: int
    arrival: float       # seconds from stream start
    env: EnvSpec
    substeps: int
    backward: bool
    loss_weights: np.ndarray


def serving_stream(seed: int = 5, rate: float = 200.0, duration: float = 60.0,
                   n_lo: int = 4000, n_hi: int = 100000,
                   max_requests: Optional[int] = None) -> List[Request]:
    """Poisson arrivals; each request is one env of a random grid, size and material."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration or (max_requests is not None and rid >= max_requests):
            break
        n = int((32, 48, 64)[int(rng.integers(0, 3))])
        N = int(rng.integers(n_lo, n_hi + 1))
        mat = MIXED_MATERIALS[int(rng.integers(0, 3))]
        S = int(rng.integers(20, 81))
        bwd = bool(rng.uniform() < 0.5)
        dx = 1.0 / n
        side = float(np.clip((N / 8.0) ** (1.0 / 3.0) * dx, 0.1, 0.6))
        lo_ok = (WALL + 1) * dx
        hi_ok = 1.0 - (WALL + 1) * dx - side
        lo = rng.uniform(lo_ok, hi_ok, size=3)
        x = uniform_points(rng, lo, np.full(3, side), N)
        v = _f32(rng.uniform(-0.5, 0.5, size=(N, 3)))
        C, F = _rest_state(N)
        env = EnvSpec(n=n, dt=5e-5, rho=1e3, Vp=side ** 3 / N, x=x, v=v, C=C, F=F, **mat)
        w = _f32(rng.standard_normal((N, 3)))
        out.append(Request(rid, t, env, S, bwd, w))
        rid += 1
    return out


WORKLOADS = {
    "single_nh": single_nh,
    "handflip_shape": handflip_shape,
    "handflip_gripper": handflip_gripper,
    "batched_corot": batched_corot,
    "uneven_mixed": uneven_mixed,
    "dam_break": dam_break,
}
