"""Seeded synthetic inputs of the FEM path: tetrahedral meshes and batches.

Input generation only (meshes, rest shapes, initial states, parameters,
activations); nothing here computes a step of the method. The tests, the
oracle checks and the bench draw their FEM inputs from here.

The paper's SoftJumper quadruped (Appendix E task table: 204 nodes, 444
tetrahedra, rho = 1, lam = mu = 1000, k_damp = 1, 80 substeps per 1/60 s
frame, initial volume scaled by U(0.9, 1.1) and the body placed at random)
is stood in for by `jumper_mesh`: a slab body on four legs cut from a cube
lattice, 199 nodes and 480 tetrahedra; the paper's own mesh asset is not
available.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Iterable, Tuple

import numpy as np

FRAME_DT = 1.0 / 60.0


def cube_lattice_mesh(cells: Iterable[Tuple[int, int, int]], h: float):
    """Nodes and tetrahedra of a union of unit lattice cubes scaled by h. Every
    cube is cut into the 6 tetrahedra around its (0,0,0)-(1,1,1) diagonal (one
    per order of the axes), so neighbouring cubes share faces exactly."""
    cells = sorted(set(tuple(int(a) for a in c) for c in cells))
    index = {}
    nodes = []

    def node(p):
        if p not in index:
            index[p] = len(nodes)
            nodes.append(p)
        return index[p]

    tets = []
    perms = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
    for c in cells:
        for perm in perms:
            p = list(c)
            path = [node(tuple(p))]
            for ax in perm:
                p[ax] += 1
                path.append(node(tuple(p)))
            tets.append(path)
    X = np.asarray(nodes, dtype=np.float64) * h
    return X, np.asarray(tets, dtype=np.int32)


def jumper_mesh(h: float = 0.05):
    """Quadruped: an 8 x 4 x 2 cube body on four 1 x 1 x 4 legs at its corners."""
    legs = [(0, 0), (7, 0), (0, 3), (7, 3)]
    cells = [(i, j, k) for i in range(8) for j in range(4) for k in range(4, 6)]
    cells += [(i, j, k) for (i, j) in legs for k in range(4)]
    return cube_lattice_mesh(cells, h)


@dataclass
class FemWorkload:
    name: str
    tets: np.ndarray      # [T, 4] int32, shared by every env
    X: np.ndarray         # [E, n, 3] float32 rest positions
    x0: np.ndarray        # [E, n, 3] float32
    v0: np.ndarray        # [E, n, 3] float32
    params: np.ndarray    # [E, 8] float64: mu, lam, rho, damp, k_e, k_d, k_f, z_g
    act: np.ndarray       # [S, E, T] float32 activations
    dt: float
    substeps: int
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.8)

    @property
    def n_envs(self) -> int:
        return self.X.shape[0]


def soft_jumper(seed: int = 7, n_envs: int = 16, substeps: int = 80, act_scale: float = 0.2,
                h: float = 0.05) -> FemWorkload:
    """A batch of jumpers (cube edge h: a 0.4 x 0.2 x 0.1 body on 0.2 legs):
    rest shape scaled by U(0.9, 1.1) per env (volume randomisation), shifted
    by U(-0.1, 0.1) in x, y and lifted by U(0, 0.02) so the feet start at or
    above the ground z = 0; at rest, at zero velocity; per-element activations
    U(-act_scale, act_scale), a new draw every frame of 80 substeps (the
    task's action is per frame); mu = lam = 1000, rho = 1, damping 1, ground
    stiffness 100, damping and friction 0.04. The explicit step is stable at
    this size: the lightest (corner) nodes' elastic and ground frequencies
    times dt stay below 2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Xm, tets = jumper_mesh(h)
    E, n, T = n_envs, Xm.shape[0], tets.shape[0]
    s = rng.uniform(0.9, 1.1, size=(E, 1, 1))
    off = np.concatenate([rng.uniform(-0.1, 0.1, size=(E, 1, 2)), rng.uniform(0.0, 0.02, size=(E, 1, 1))], axis=2)
    X = (Xm[None] * s + off).astype(np.float32)
    prm = np.tile(np.array([1000.0, 1000.0, 1.0, 1.0, 100.0, 0.04, 0.04, 0.0]), (E, 1))
    frames = -(-substeps // 80)
    per_frame = rng.uniform(-act_scale, act_scale, size=(frames, E, T))
    act = np.repeat(per_frame, 80, axis=0)[:substeps].astype(np.float32)
    return FemWorkload("soft_jumper", tets, X, X.copy(), np.zeros_like(X), prm, act, FRAME_DT / 80.0, substeps)


def two_cubes(seed: int = 3, n_envs: int = 3, substeps: int = 12, h: float = 0.05) -> FemWorkload:
    """A small case: two stacked cubes (12 nodes, 12 tetrahedra), each env
    stretched, sheared and moving at random, half of them touching the ground."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Xm, tets = cube_lattice_mesh([(0, 0, 0), (0, 0, 1)], h)
    E, n, T = n_envs, Xm.shape[0], tets.shape[0]
    X = (Xm[None] + rng.uniform(-0.2, 0.2, size=(E, 1, 3)) * np.array([1, 1, 0]) + 0.01).astype(np.float32)
    A = np.eye(3)[None] + rng.uniform(-0.15, 0.15, size=(E, 3, 3))
    x0 = np.einsum("eij,enj->eni", A, X - X.mean(1, keepdims=True)) + X.mean(1, keepdims=True)
    x0[:, :, 2] -= np.where(np.arange(E) % 2 == 0, 0.015, 0.0)[:, None]   # even envs press into the ground
    v0 = rng.uniform(-0.3, 0.3, size=(E, n, 3))
    prm = np.column_stack([rng.uniform(500, 1500, E), rng.uniform(500, 2000, E), rng.uniform(0.5, 2.0, E),
                           rng.uniform(0.0, 2.0, E), np.full(E, 200.0), np.full(E, 0.1), np.full(E, 0.1),
                           np.zeros(E)])
    act = rng.uniform(-0.2, 0.2, size=(substeps, E, T)).astype(np.float32)
    return FemWorkload("two_cubes", tets, X, x0.astype(np.float32), v0.astype(np.float32), prm, act, 1e-4, substeps)
