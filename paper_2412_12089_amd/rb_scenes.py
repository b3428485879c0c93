"""Seeded synthetic inputs of the articulated rigid-body path: link trees and batches.

Input generation only (link geometry and inertia, initial states, torques,
parameters); nothing here steps the dynamics. The paper's rigid-body tasks
drive a robot hand and a quadruped whose assets are not available; `hand`
stands in for a fixed-base hand: a palm on a wrist joint and fingers of
three links each, with contact spheres at the finger tips.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

FRAME_DT = 1.0 / 60.0


@dataclass
class RbLink:
    parent: int
    joint_pos: np.ndarray
    joint_rot: np.ndarray
    axis: np.ndarray
    mass: float
    com: np.ndarray
    inertia: np.ndarray
    contacts: List[Tuple[np.ndarray, float]]
    joint: str = "revolute"     # or "prismatic": the link slides along the axis


def rod_inertia(mass: float, length: float, radius: float, axis: int) -> np.ndarray:
    """Solid cylinder about its centre, long along `axis`."""
    I = np.full(3, mass * (3 * radius ** 2 + length ** 2) / 12.0)
    I[axis] = 0.5 * mass * radius ** 2
    return np.diag(I)


def rot_about(axis, angle) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def pendulum(length: float = 0.5, mass: float = 1.0) -> List[RbLink]:
    """One link hanging from a hinge about x, its mass at the end."""
    return [RbLink(-1, np.zeros(3), np.eye(3), np.array([1.0, 0, 0]), mass, np.array([0, 0, -length]),
                   np.eye(3) * 1e-4, [])]


def two_link_arm(l1=0.6, l2=0.4, m1=1.5, m2=0.8) -> List[RbLink]:
    """Planar arm in the y-z plane (hinges about x), point-like masses at the link ends."""
    return [RbLink(-1, np.zeros(3), np.eye(3), np.array([1.0, 0, 0]), m1, np.array([0, 0, -l1]),
                   np.zeros((3, 3)), []),
            RbLink(0, np.array([0, 0, -l1]), np.eye(3), np.array([1.0, 0, 0]), m2, np.array([0, 0, -l2]),
                   np.zeros((3, 3)), [])]


def cart_pole(m_cart: float = 1.2, m_pole: float = 0.4, l: float = 0.5) -> List[RbLink]:
    """A cart sliding along x (prismatic) carrying a pole hinged about y, a point-like mass at distance l
    along the pole's -z axis."""
    return [RbLink(-1, np.zeros(3), np.eye(3), np.array([1.0, 0, 0]), m_cart, np.zeros(3), np.zeros((3, 3)), [],
                   joint="prismatic"),
            RbLink(0, np.zeros(3), np.eye(3), np.array([0, 1.0, 0]), m_pole, np.array([0, 0, -l]), np.zeros((3, 3)),
                   [])]


def hand(n_fingers: int = 4, seg: Tuple[float, ...] = (0.05, 0.035, 0.025), palm: float = 0.09,
         height: float = 0.12) -> List[RbLink]:
    """A palm turning about the vertical on a wrist at `height`, and fingers of
    len(seg) links bending about the palm's x axis (the first joint of each
    finger also splays about the palm normal), a contact sphere at each tip."""
    links: List[RbLink] = []
    links.append(RbLink(-1, np.array([0.0, 0.0, height]), np.eye(3), np.array([0.0, 0, 1.0]), 0.3,
                        np.array([0, palm / 2, 0]), np.diag([4e-4, 1e-4, 4e-4]), []))
    for f in range(n_fingers):
        x0 = (f - (n_fingers - 1) / 2) * 0.025
        parent = 0
        for k, L in enumerate(seg):
            pos = np.array([x0, palm, 0.0]) if k == 0 else np.array([0.0, seg[k - 1], 0.0])
            jr = rot_about([0, 0, 1], 0.15 * (f - (n_fingers - 1) / 2)) if k == 0 else np.eye(3)
            m = 0.04 * L / 0.05
            tip = [(np.array([0.0, L, 0.0]), 0.008)] if k == len(seg) - 1 else []
            links.append(RbLink(parent, pos, jr, np.array([1.0, 0, 0]), m, np.array([0, L / 2, 0]),
                                rod_inertia(m, L, 0.007, 1), tip))
            parent = len(links) - 1
    return links


@dataclass
class RbWorkload:
    name: str
    links: List[RbLink]
    q0: np.ndarray       # [E, N] float32
    qd0: np.ndarray      # [E, N] float32
    params: np.ndarray   # [E, 5] float64: damp, k_e, k_d, k_f, z_g
    tau: np.ndarray      # [S, E, N] float32 joint torques
    dt: float
    substeps: int
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.8)

    @property
    def n_envs(self) -> int:
        return self.q0.shape[0]


def hand_batch(seed: int = 9, n_envs: int = 8, substeps: int = 16, n_fingers: int = 4,
               torque: float = 2e-3, dt: float = FRAME_DT / 16) -> RbWorkload:
    """Hands (wrist at z = 0.12) at random joint angles and speeds over a
    ground at z_g = 0.095 that the finger tips reach when they bend down (about
    one tip in ten touches it at any time), joint damping U(1e-5, 1e-4),
    ground stiffness 200, damping 1, friction 0.5, and torques U(-torque,
    torque) drawn per frame and held over the frame's substeps. The finger
    links weigh 10-40 g, so torques and damping are of the order of their
    gravity torques."""
    rng = np.random.Generator(np.random.PCG64(seed))
    links = hand(n_fingers)
    N = len(links)
    q0 = rng.uniform(-0.6, 0.9, size=(n_envs, N))
    q0[:, 0] = rng.uniform(-0.5, 0.5, n_envs)
    qd0 = rng.uniform(-1.0, 1.0, size=(n_envs, N))
    prm = np.column_stack([rng.uniform(1e-5, 1e-4, n_envs), np.full(n_envs, 200.0), np.full(n_envs, 1.0),
                           np.full(n_envs, 0.5), np.full(n_envs, 0.095)])
    frames = -(-substeps // 16)
    per = rng.uniform(-torque, torque, size=(frames, n_envs, N))
    tau = np.repeat(per, 16, axis=0)[:substeps]
    return RbWorkload("hand", links, q0.astype(np.float32), qd0.astype(np.float32), prm, tau.astype(np.float32), dt,
                      substeps)


def random_tree(seed: int, n_links: int, chain: float = 0.5, n_contacts: int = 4,
                prismatic: float = 0.0) -> List[RbLink]:
    """A random tree of n_links links: each link hangs from a random earlier
    one (from the one just before it with probability `chain`), with a random
    joint frame and axis, 0.1-1 kg, a centre of mass 5-20 cm out and a random
    positive definite inertia; contact spheres on the last n_contacts links.
    Joints are revolute, or prismatic with probability `prismatic` (drawn
    after the rest of the tree, so the other draws do not depend on it)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    links: List[RbLink] = []
    for i in range(n_links):
        parent = -1 if i == 0 else (i - 1 if rng.uniform() < chain else int(rng.integers(0, i)))
        pos = np.array([0.0, 0.0, 0.5]) if i == 0 else rng.uniform(-0.15, 0.15, 3)
        jr = rot_about(rng.standard_normal(3), rng.uniform(-np.pi, np.pi))
        ax = rng.standard_normal(3)
        ax /= np.linalg.norm(ax)
        m = rng.uniform(0.1, 1.0)
        com = rng.uniform(-0.2, 0.2, 3)
        com *= rng.uniform(0.05, 0.2) / np.linalg.norm(com)
        Q = rot_about(rng.standard_normal(3), rng.uniform(0, np.pi))
        I = Q @ np.diag(m * rng.uniform(2e-3, 1e-2, 3)) @ Q.T
        cts = [(com * 1.5, 0.02)] if i >= n_links - n_contacts else []
        links.append(RbLink(parent, pos, jr, ax, m, com, I, cts))
    if prismatic > 0.0:
        kinds = np.random.Generator(np.random.PCG64(seed + 7)).uniform(size=n_links)
        for L, u in zip(links, kinds):
            if u < prismatic:
                L.joint = "prismatic"
    return links


def tree_batch(seed: int, n_links: int, n_envs: int = 4, substeps: int = 6, dt: float = FRAME_DT / 16,
               ground: float = 0.3, n_contacts: int = 4, roots: int = 1, prismatic: float = 0.0) -> RbWorkload:
    """Random states (angles U(-1, 1), speeds U(-2, 2)) and torques U(-0.5, 0.5)
    on `random_tree`, joint damping U(0.01, 0.05), a ground at z_g = `ground`
    with stiffness 2000. With roots > 1 the links are split into that many
    trees (a forest: link k * n_links // roots starts a new tree)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    links = random_tree(seed, n_links, n_contacts=n_contacts, prismatic=prismatic)
    for r in range(1, roots):
        k = r * n_links // roots
        links[k].parent = -1
        links[k].joint_pos = np.array([0.4 * r, 0.0, 0.5])
        for i in range(k + 1, n_links):
            if links[i].parent < k:
                links[i].parent = k if links[i].parent >= 0 else -1
        for i in range(k + 1, n_links):
            if links[i].parent == -1:
                links[i].parent = k
    N = len(links)
    q0 = rng.uniform(-1.0, 1.0, size=(n_envs, N))
    qd0 = rng.uniform(-2.0, 2.0, size=(n_envs, N))
    prm = np.column_stack([rng.uniform(0.01, 0.05, n_envs), np.full(n_envs, 2000.0), np.full(n_envs, 5.0),
                           np.full(n_envs, 1.0), np.full(n_envs, ground)])
    tau = rng.uniform(-0.5, 0.5, size=(substeps, n_envs, N))
    return RbWorkload(f"tree{n_links}", links, q0.astype(np.float32), qd0.astype(np.float32), prm,
                      tau.astype(np.float32), dt, substeps)
