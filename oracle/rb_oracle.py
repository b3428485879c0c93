"""FP64 CPU oracle of the batched articulated rigid-body step.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference that the
HIP rigid-body path is checked against. Only the test suite, the smoke check
and the bench's CPU-baseline leg may import it; the library never calls it.

Appendix D.1 (composite rigid body algorithm) writes the articulated dynamics
as M(q) qdd = J^T F(q, qd) + c(q, qd) + tau, solved for the joint
accelerations and stepped by semi-implicit Euler. This oracle does not run
the composite rigid body algorithm or any recursion over the tree: it writes
the same dynamics from their definition, Lagrange's equations of the tree's
kinetic and potential energy, so that the two routes check each other:
    T(q, qd) = 1/2 qd^T M(q) qd,  M = sum_i m_i Jc_i^T Jc_i + Jw_i^T I_i^world Jw_i,
    V(q) = - sum_i m_i g . c_i,
    bias = (d/dq dT/dqd) qd - dT/dq + dV/dq            (Coriolis, centrifugal, gravity),
    M qdd = tau - bias - damp qd + Q_contact,
    qd' = qd + dt qdd,  q' = q + dt qd'.
Jc_i and Jw_i are the geometric Jacobians of body i's centre of mass and of
its angular velocity; the second derivatives of T come from automatic
differentiation.

Readings (each listed in the design notes): every joint is a revolute joint
about a body-fixed axis through the joint origin, or a prismatic joint
sliding along one, on a fixed base (the robot hands' case); joint damping is viscous, -damp qd; contact is the ground
half-space z >= z_g acting on spheres fixed to the bodies, at the lowest point
of each sphere, with normal force k_e (z_g - z) - k_d v_z and viscous friction
-k_f v_t while that point is below z_g, v the velocity of the body's material
point there; it enters the joints as the generalised force J^T f.

Kinematics: body i's frame is its joint frame (placed in the parent body's
frame by a fixed rotation Rt_i and offset pt_i; in the world for a root)
turned by q_i about the joint axis a_i: R_i = R_parent Rt_i Rot(a_i, q_i),
p_i = p_parent + R_parent pt_i; or, for a prismatic joint, slid by q_i along
it: R_i = R_parent Rt_i, p_i = p_parent + R_parent (pt_i + Rt_i a_i q_i).
A revolute joint j moves a point x of a body below it at w_j x (x - o_j) per
unit qd_j and turns the body at w_j (w_j the world joint axis, o_j the joint
origin); a prismatic one moves it at w_j and turns nothing.

Every function takes a batch of environments: q, qd, tau [E, N], params
[E, 5] (damp, k_e, k_d, k_f, z_g); the links are shared.
"""
from __future__ import annotations

from typing import List

import numpy as np
import torch

DT = torch.float64
RB_PARAMS = ("damp", "ke", "kd", "kf", "ground")


def _t(a):
    if torch.is_tensor(a):
        return a.to(DT)
    return torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=DT)


def rot(axis, angle):
    """Rotation by angle [E] about the unit axis [3] (Rodrigues): [E, 3, 3]."""
    a = _t(axis)
    K = torch.zeros(3, 3, dtype=DT)
    K[0, 1], K[0, 2], K[1, 0], K[1, 2], K[2, 0], K[2, 1] = -a[2], a[1], a[2], -a[0], -a[1], a[0]
    s, c = torch.sin(angle)[:, None, None], torch.cos(angle)[:, None, None]
    return torch.eye(3, dtype=DT) + s * K + (1.0 - c) * (K @ K)


def prismatic(L) -> bool:
    return getattr(L, "joint", "revolute") == "prismatic"


def kinematics(links, q):
    """World rotation [E, 3, 3] and origin [E, 3] of every body frame."""
    E = q.shape[0]
    R, p = [], []
    for i, L in enumerate(links):
        if L.parent < 0:
            Rp, pp = torch.eye(3, dtype=DT).expand(E, 3, 3), torch.zeros(E, 3, dtype=DT)
        else:
            Rp, pp = R[L.parent], p[L.parent]
        Rt = _t(L.joint_rot)
        if prismatic(L):
            R.append(Rp @ Rt)
            p.append(pp + Rp @ _t(L.joint_pos) + q[:, i:i + 1] * (Rp @ (Rt @ _t(L.axis))))
        else:
            R.append(Rp @ Rt @ rot(L.axis, q[:, i]))
            p.append(pp + Rp @ _t(L.joint_pos))
    return R, p


def ancestors(links, i: int) -> List[int]:
    """Joints on the path from the root to body i, body i's own joint included."""
    out = []
    while i >= 0:
        out.append(i)
        i = links[i].parent
    return out[::-1]


def world_axis(links, R, j):
    """World joint axis w_j [E, 3] (the joint turns about its own axis, so R_j a_j)."""
    return R[j] @ _t(links[j].axis)


def point_jacobian(links, R, p, i: int, x):
    """d x / d q [E, 3, N] of a point x [E, 3] fixed to body i: column j (a
    joint above the body) is w_j x (x - o_j), or w_j for a prismatic joint;
    other columns are zero."""
    E, N = x.shape[0], len(links)
    cols = [torch.zeros(E, 3, dtype=DT)] * N
    for j in ancestors(links, i):
        w = world_axis(links, R, j)
        cols[j] = w.expand(E, 3) if prismatic(links[j]) else torch.linalg.cross(w, x - p[j])
    return torch.stack(cols, dim=2)


def angular_jacobian(links, R, i: int):
    """d w_i / d qd [E, 3, N]: column j (a revolute joint above the body) is
    w_j; a prismatic joint turns nothing."""
    E, N = R[0].shape[0], len(links)
    cols = [torch.zeros(E, 3, dtype=DT)] * N
    for j in ancestors(links, i):
        if not prismatic(links[j]):
            cols[j] = world_axis(links, R, j)
    return torch.stack(cols, dim=2)


def com(links, R, p, i):
    return p[i] + R[i] @ _t(links[i].com)


def mass_matrix(links, q):
    """M(q) [E, N, N] = sum_i m_i Jc_i^T Jc_i + Jw_i^T (R_i I_i R_i^T) Jw_i, the
    matrix of the kinetic energy's quadratic form."""
    R, p = kinematics(links, q)
    M = 0
    for i, L in enumerate(links):
        Jc = point_jacobian(links, R, p, i, com(links, R, p, i))
        Jw = angular_jacobian(links, R, i)
        Iw = R[i] @ _t(L.inertia) @ R[i].transpose(1, 2)
        M = M + L.mass * Jc.transpose(1, 2) @ Jc + Jw.transpose(1, 2) @ Iw @ Jw
    return M


def kinetic(links, q, qd):
    """T [E] = 1/2 qd^T M(q) qd."""
    return 0.5 * torch.einsum("ei,eij,ej->e", qd, mass_matrix(links, q), qd)


def potential(links, q, gravity):
    """V [E] = - sum_i m_i g . c_i."""
    R, p = kinematics(links, q)
    g = _t(gravity)
    return -sum(L.mass * (com(links, R, p, i) @ g) for i, L in enumerate(links))


def bias(links, q, qd, gravity):
    """Lagrange's equations without the acceleration term [E, N]:
    sum_j d^2T/(dqd_k dq_j) qd_j - dT/dq_k + dV/dq_k. The first term is the
    qd-gradient of dT/dq . u with u = qd held fixed; q and qd enter T as
    separate copies so that outer derivatives still see every dependence."""
    with torch.enable_grad():
        qa = q.clone() if q.requires_grad else q.detach().clone().requires_grad_(True)
        qda = qd.clone() if qd.requires_grad else qd.detach().clone().requires_grad_(True)
        T = kinetic(links, qa, qda).sum()
        dT_dq = torch.autograd.grad(T, qa, create_graph=True)[0]
        term1 = torch.autograd.grad((dT_dq * qd).sum(), qda, create_graph=True)[0]
        dV_dq = torch.autograd.grad(potential(links, qa, gravity).sum(), qa, create_graph=True)[0]
    return term1 - dT_dq + dV_dq


def contact_points(links, R, p):
    """(body, world point [E, 3]) of the lowest point of every contact sphere."""
    out = []
    for i, L in enumerate(links):
        for (c, r) in L.contacts:
            out.append((i, p[i] + R[i] @ _t(c) - float(r) * _t([0.0, 0.0, 1.0])))
    return out


def contact_force(links, q, qd, prm):
    """Generalised ground force [E, N]: J^T f summed over the contact spheres,
    f the penalty force at each sphere's lowest point while it is below z_g."""
    ke, kd, kf, zg = prm[:, 1:2], prm[:, 2:3], prm[:, 3:4], prm[:, 4]
    R, p = kinematics(links, q)
    Q = torch.zeros_like(q)
    for i, x in contact_points(links, R, p):
        J = point_jacobian(links, R, p, i, x)
        vel = (J @ qd[:, :, None])[:, :, 0]
        depth = zg - x[:, 2]
        f = torch.cat([-kf * vel[:, :2], ke * depth[:, None] - kd * vel[:, 2:3]], dim=1)
        Q = Q + torch.where((depth > 0)[:, None], (J.transpose(1, 2) @ f[:, :, None])[:, :, 0], 0.0)
    return Q


def accel(links, q, qd, tau, prm, gravity):
    """qdd [E, N] = M^-1 (tau - bias - damp qd + Q_contact)."""
    rhs = tau - bias(links, q, qd, gravity) - prm[:, 0:1] * qd + contact_force(links, q, qd, prm)
    return torch.linalg.solve(mass_matrix(links, q), rhs)


def step(links, q, qd, tau, prm, gravity, dt):
    qd1 = qd + dt * accel(links, q, qd, tau, prm, gravity)
    return q + dt * qd1, qd1


def rollout(links, q0, qd0, tau, prm, gravity, dt, S, keep_all=False):
    """S substeps from (q0, qd0) [E, N] under tau [>= S, E, N]."""
    q, qd, tau, prm = (_t(a) for a in (q0, qd0, tau, prm))
    track = any(t.requires_grad or _is_dual(t) for t in (q, qd, tau, prm))
    states = [(q, qd)]
    for k in range(S):
        q, qd = step(links, q, qd, tau[k], prm, gravity, dt)
        if not track:
            q, qd = q.detach(), qd.detach()
        if keep_all:
            states.append((q, qd))
    return (q, qd, states) if keep_all else (q, qd)


def _is_dual(t):
    import torch.autograd.forward_ad as fwAD
    return fwAD.unpack_dual(t).tangent is not None


def rollout_vjp(links, q0, qd0, tau, prm, gravity, dt, S, gq, gqd):
    """Cotangents of (q0, qd0, tau[:S], params) for cotangents (gq, gqd) of the
    final state, by reverse-mode autograd through the rollout as written."""
    q0, qd0, prm = (_t(a).clone().requires_grad_(True) for a in (q0, qd0, prm))
    tau = _t(tau)[:S].clone().requires_grad_(True)
    q, qd = rollout(links, q0, qd0, tau, prm, gravity, dt, S)
    L = (q * _t(gq)).sum() + (qd * _t(gqd)).sum()
    g = torch.autograd.grad(L, (q0, qd0, tau, prm), allow_unused=True)
    return tuple(torch.zeros_like(t) if gi is None else gi.detach() for gi, t in zip(g, (q0, qd0, tau, prm)))
