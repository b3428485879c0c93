"""Pins of the rigid-body oracle (oracle/rb_oracle.py) to what mechanics fixes,
independently of the oracle's own formulas (CPU only).

Appendix D.1: articulated bodies, M(q) qdd = J^T F + c + tau, semi-implicit
Euler. The pins: textbook mass matrices and Lagrange equations of a pendulum,
a planar two-link arm, a spherical pendulum and a symmetric top on a gimbal;
the mass matrix against the Hessian of a kinetic energy built from velocities
obtained by differentiating the kinematics in time; the power balance and a
conserved momentum of the exact dynamics; a contact force worked by hand; the
reverse-mode gradients of a rollout against central differences.
"""
import math

import numpy as np
import pytest
import torch

from oracle import rb_oracle as RO
from paper_2412_12089_amd import rb_scenes as RS

DT64 = torch.float64
G = 9.8
NO_GROUND = [0.0, 0.0, 0.0, 0.0, -1e9]


def t64(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def link(parent, pos, axis, mass, com, inertia, contacts=()):
    return RS.RbLink(parent, np.asarray(pos, float), np.eye(3), np.asarray(axis, float), mass,
                     np.asarray(com, float), np.asarray(inertia, float), list(contacts))


def test_pendulum_closed_form():
    """One hinge, point-like mass m at distance l plus inertia I about the
    hinge axis through the COM: M = m l^2 + I, bias = m g l sin q, no velocity
    term (one degree of freedom)."""
    m, l, Ixx = 1.3, 0.7, 0.02
    L = [link(-1, [0, 0, 0], [1, 0, 0], m, [0, 0, -l], np.diag([Ixx, 0.01, 0.03]))]
    q = t64([[0.4], [-1.1], [2.5]])
    qd = t64([[0.0], [3.0], [-2.0]])
    M = RO.mass_matrix(L, q)
    assert torch.allclose(M[:, 0, 0], torch.full((3,), m * l * l + Ixx, dtype=DT64), rtol=1e-13)
    b = RO.bias(L, q, qd, (0.0, 0.0, -G))
    assert torch.allclose(b[:, 0], m * G * l * torch.sin(q[:, 0]), rtol=1e-12, atol=1e-13)
    qdd = RO.accel(L, q, qd, torch.zeros_like(q), t64([NO_GROUND] * 3), (0.0, 0.0, -G))
    assert torch.allclose(qdd[:, 0], -m * G * l * torch.sin(q[:, 0]) / (m * l * l + Ixx), rtol=1e-12)


def test_two_link_arm_textbook():
    """Planar arm with point masses at the link ends (hinges about x, angles
    from the downward vertical, the second relative to the first):
    M11 = m1 l1^2 + m2 (l1^2 + l2^2 + 2 l1 l2 c2), M12 = m2 (l2^2 + l1 l2 c2), M22 = m2 l2^2,
    b1 = -m2 l1 l2 s2 (2 qd1 qd2 + qd2^2) + (m1 + m2) g l1 s1 + m2 g l2 s12,
    b2 = m2 l1 l2 s2 qd1^2 + m2 g l2 s12."""
    l1, l2, m1, m2 = 0.6, 0.4, 1.5, 0.8
    L = RS.two_link_arm(l1, l2, m1, m2)
    rng = np.random.default_rng(0)
    q = t64(rng.uniform(-2, 2, (5, 2)))
    qd = t64(rng.uniform(-3, 3, (5, 2)))
    M = RO.mass_matrix(L, q).numpy()
    b = RO.bias(L, q, qd, (0.0, 0.0, -G)).detach().numpy()
    for e in range(5):
        q1, q2 = q[e].numpy()
        d1, d2 = qd[e].numpy()
        c2, s2 = math.cos(q2), math.sin(q2)
        Mt = np.array([[m1 * l1 ** 2 + m2 * (l1 ** 2 + l2 ** 2 + 2 * l1 * l2 * c2), m2 * (l2 ** 2 + l1 * l2 * c2)],
                       [m2 * (l2 ** 2 + l1 * l2 * c2), m2 * l2 ** 2]])
        bt = np.array([-m2 * l1 * l2 * s2 * (2 * d1 * d2 + d2 * d2) + (m1 + m2) * G * l1 * math.sin(q1)
                       + m2 * G * l2 * math.sin(q1 + q2),
                       m2 * l1 * l2 * s2 * d1 * d1 + m2 * G * l2 * math.sin(q1 + q2)])
        np.testing.assert_allclose(M[e], Mt, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(b[e], bt, rtol=1e-11, atol=1e-12)


def test_spherical_pendulum_and_symmetric_top():
    """Azimuth phi about z, then polar angle theta about the turned x axis; the
    second body has a point-like mass m at distance l below the pivot plus a
    rotational inertia diag(A, A, C) (symmetric about its own z axis):
    T = 1/2 (m l^2 + A) thd^2 + 1/2 ((m l^2 + A) s^2 + C c^2) phd^2,  V = -m g l c,
    so M = diag((m l^2 + A) s^2 + C c^2, m l^2 + A) and Lagrange's equations give
    b_phi = 2 (m l^2 + A - C) s c thd phd,  b_theta = -(m l^2 + A - C) s c phd^2 + m g l s."""
    m, l, A, C = 0.9, 0.5, 0.03, 0.05
    L = [link(-1, [0, 0, 0], [0, 0, 1], 0.0, [0, 0, 0], np.zeros((3, 3))),
         link(0, [0, 0, 0], [1, 0, 0], m, [0, 0, -l], np.diag([A, A, C]))]
    rng = np.random.default_rng(1)
    q = t64(np.column_stack([rng.uniform(-3, 3, 6), rng.uniform(0.3, 2.8, 6)]))
    qd = t64(rng.uniform(-2, 2, (6, 2)))
    M = RO.mass_matrix(L, q).numpy()
    b = RO.bias(L, q, qd, (0.0, 0.0, -G)).detach().numpy()
    K = m * l * l + A
    for e in range(6):
        th = q[e, 1].item()
        s, c = math.sin(th), math.cos(th)
        dphi, dth = qd[e].numpy()
        np.testing.assert_allclose(M[e], np.diag([K * s * s + C * c * c, K]), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(b[e], [2 * (K - C) * s * c * dth * dphi,
                                          -(K - C) * s * c * dphi ** 2 + m * G * l * s], rtol=1e-11, atol=1e-12)


def _kinetic_from_motion(links, q, qd):
    """Kinetic energy from velocities taken as time derivatives of the
    kinematics along qd (forward mode), not from Jacobians:
    sum_i 1/2 m_i |dc_i/dt|^2 + 1/2 w_i . (R_i I_i R_i^T) w_i, [w_i]x = dR_i/dt R_i^T."""
    def poses(qq):
        R, p = RO.kinematics(links, qq)
        cs = [p[i] + R[i] @ RO._t(L.com) for i, L in enumerate(links)]
        return tuple(R) + tuple(cs)
    _, dots = torch.autograd.functional.jvp(poses, q, qd, create_graph=True)
    R, p = RO.kinematics(links, q)
    n = len(links)
    T = 0
    for i, L in enumerate(links):
        cdot = dots[n + i]
        W = dots[i] @ R[i].transpose(1, 2)
        w = torch.stack([W[:, 2, 1], W[:, 0, 2], W[:, 1, 0]], dim=1)
        Iw = R[i] @ RO._t(L.inertia) @ R[i].transpose(1, 2)
        T = T + 0.5 * L.mass * (cdot * cdot).sum(1) + 0.5 * torch.einsum("ei,eij,ej->e", w, Iw, w)
    return T


def test_mass_matrix_is_hessian_of_motion_energy():
    """On the hand: M equals the Hessian in qd of the kinetic energy built from
    differentiated kinematics, and M is symmetric positive definite."""
    wl = RS.hand_batch(seed=2, n_envs=2)
    L = wl.links
    q = t64(wl.q0)
    M = RO.mass_matrix(L, q)
    for e in range(2):
        H = torch.autograd.functional.hessian(
            lambda qd: _kinetic_from_motion(L, q[e:e + 1], qd[None])[0], torch.zeros(len(L), dtype=DT64))
        assert torch.allclose(M[e], H, rtol=1e-10, atol=1e-14)
        assert torch.allclose(M[e], M[e].T, rtol=0, atol=1e-18)
        assert torch.linalg.eigvalsh(M[e]).min() > 0


def test_power_balance():
    """d(T + V)/dt = qd . (tau - damp qd + Q_contact) along the exact dynamics,
    at hand states with contacts, torques and damping active."""
    wl = RS.hand_batch(seed=3, n_envs=4)
    L = wl.links
    prm = t64(wl.params)
    prm[:, 4] = 0.118                      # a ground just under the palm: finger tips touch it
    prm[:, 0] = 0.02
    q, qd, tau = t64(wl.q0), t64(wl.qd0), t64(wl.tau[0]) * 10
    Qc = RO.contact_force(L, q, qd, prm)
    assert (Qc.abs().sum(1) > 0).sum() >= 3
    qdd = RO.accel(L, q, qd, tau, prm, wl.gravity).detach()
    qa, qda = q.clone().requires_grad_(True), qd.clone().requires_grad_(True)
    E = (RO.kinetic(L, qa, qda) + RO.potential(L, qa, wl.gravity)).sum()
    gq, gqd = torch.autograd.grad(E, (qa, qda))
    dE = (gq * qd).sum(1) + (gqd * qdd).sum(1)
    power = (qd * (tau - prm[:, 0:1] * qd + Qc)).sum(1)
    assert torch.allclose(dE, power, rtol=1e-9, atol=1e-12)


def test_cyclic_wrist_momentum():
    """With gravity along the wrist's vertical axis and no ground, no torque and
    no damping, the wrist angle is a cyclic coordinate: its momentum (M qd)_0
    has zero time derivative, dM/dt qd + M qdd = 0 in row 0."""
    wl = RS.hand_batch(seed=4, n_envs=3)
    L = wl.links
    q, qd = t64(wl.q0), t64(wl.qd0)
    prm = t64([NO_GROUND] * 3)
    qdd = RO.accel(L, q, qd, torch.zeros_like(q), prm, wl.gravity).detach()
    h = 1e-6
    Mdot = (RO.mass_matrix(L, q + h * qd) - RO.mass_matrix(L, q - h * qd)) / (2 * h)
    M = RO.mass_matrix(L, q)
    dp = (Mdot @ qd[:, :, None] + M @ qdd[:, :, None])[:, 0, 0]
    scale = (M @ qdd[:, :, None]).abs()[:, :, 0].max()
    assert dp.abs().max() < 1e-7 * scale
    # while the fingers' own momenta do change
    assert (Mdot @ qd[:, :, None] + M @ qdd[:, :, None])[:, 1:, 0].abs().max() > 1e-3 * scale


def test_contact_hand_value():
    """A pendulum hinged about x at height h with a contact sphere (radius r)
    at its end, dipped below the ground: the lowest point is
    x = (0, l s, h - l c - r), moving at qd (0, l c + r, l s) (the material
    point there), the force f = (0, -k_f v_y, k_e (z_g - x_z) - k_d v_z) and the
    joint torque (x - o) x f . e_x = l s f_z + (l c + r) f_y."""
    h, l, r, q0, qd0 = 0.3, 0.35, 0.02, 0.4, -1.2
    ke, kd, kf, zg = 500.0, 3.0, 0.7, 0.0
    L = [link(-1, [0, 0, h], [1, 0, 0], 1.0, [0, 0, -l], np.eye(3) * 1e-3, [(np.array([0, 0, -l]), r)])]
    s, c = math.sin(q0), math.cos(q0)
    xz = h - l * c - r
    assert xz < zg
    vy, vz = qd0 * (l * c + r), qd0 * l * s
    fy, fz = -kf * vy, ke * (zg - xz) - kd * vz
    Q = RO.contact_force(L, t64([[q0]]), t64([[qd0]]), t64([[0.0, ke, kd, kf, zg]]))
    assert Q[0, 0].item() == pytest.approx(l * s * fz + (l * c + r) * fy, rel=1e-13)
    # above the ground: nothing
    Q = RO.contact_force(L, t64([[q0]]), t64([[qd0]]), t64([[0.0, ke, kd, kf, xz - 1e-3]]))
    assert Q[0, 0].item() == 0.0


def test_rollout_vjp_central_differences():
    """Reverse-mode cotangents of a hand rollout (contacts, damping, torques)
    against central differences of the forward in random directions."""
    wl = RS.hand_batch(seed=5, n_envs=2, substeps=6)
    L = wl.links
    prm = wl.params.copy()
    prm[:, 4] = 0.07
    rng = np.random.default_rng(6)
    E, N = wl.q0.shape
    gq, gqd = rng.standard_normal((E, N)), rng.standard_normal((E, N))
    args = [wl.q0.astype(np.float64), wl.qd0.astype(np.float64), wl.tau.astype(np.float64), prm]
    grads = RO.rollout_vjp(L, *args[:3], prm, wl.gravity, wl.dt, wl.substeps, gq, gqd)

    def f(a):
        q, qd = RO.rollout(L, a[0], a[1], a[2], a[3], wl.gravity, wl.dt, wl.substeps)
        return float((q.numpy() * gq).sum() + (qd.numpy() * gqd).sum())

    scales = [1.0, 1.0, 1e-2, np.array([1e-5, 100.0, 1.0, 0.5, 0.01])]
    for k in range(4):
        d = rng.standard_normal(args[k].shape) * scales[k]
        eps = 1e-6
        ap = [a.copy() for a in args]
        am = [a.copy() for a in args]
        ap[k] = ap[k] + eps * d
        am[k] = am[k] - eps * d
        fd = (f(ap) - f(am)) / (2 * eps)
        an = float((grads[k].numpy() * d).sum())
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), k


def test_free_fall_of_released_wrist():
    """A single body on a vertical hinge with gravity along the hinge: no torque
    from gravity, so under a constant torque the angle follows the closed form
    of semi-implicit Euler, q_k = q0 + dt^2 a k (k + 1) / 2 with a = tau / I_zz."""
    Izz = 0.05
    L = [link(-1, [0, 0, 0], [0, 0, 1], 2.0, [0, 0, 0.3], np.diag([0.1, 0.2, Izz]))]
    dt, S, tau = 0.01, 7, 0.4
    q, qd = RO.rollout(L, [[0.2]], [[0.0]], np.full((S, 1, 1), tau), [NO_GROUND], (0.0, 0.0, -G), dt, S)
    a = tau / Izz
    assert q[0, 0].item() == pytest.approx(0.2 + dt * dt * a * S * (S + 1) / 2, rel=1e-13)
    assert qd[0, 0].item() == pytest.approx(dt * a * S, rel=1e-13)


def test_cart_pole_textbook():
    """A cart sliding along x (prismatic joint) carrying a pole hinged about y
    with a point mass m_p at distance l below the hinge: the pole's mass sits
    at (x - l s, 0, -l c), so T = 1/2 (m_c + m_p) xd^2 - m_p l c xd thd + 1/2 m_p l^2 thd^2
    and V = -m_p g l c, giving M = [[m_c + m_p, -m_p l c], [-m_p l c, m_p l^2]],
    b_x = m_p l s thd^2, b_theta = m_p g l s."""
    mc, mp, l = 1.2, 0.4, 0.5
    L = RS.cart_pole(mc, mp, l)
    rng = np.random.default_rng(11)
    q = t64(np.column_stack([rng.uniform(-1, 1, 6), rng.uniform(-3, 3, 6)]))
    qd = t64(rng.uniform(-2, 2, (6, 2)))
    M = RO.mass_matrix(L, q).numpy()
    b = RO.bias(L, q, qd, (0.0, 0.0, -G)).detach().numpy()
    qdd = RO.accel(L, q, qd, torch.zeros_like(q), t64([NO_GROUND] * 6), (0.0, 0.0, -G)).detach().numpy()
    for e in range(6):
        th, dth = q[e, 1].item(), qd[e, 1].item()
        s, c = math.sin(th), math.cos(th)
        Mt = np.array([[mc + mp, -mp * l * c], [-mp * l * c, mp * l * l]])
        bt = np.array([mp * l * s * dth * dth, mp * G * l * s])
        np.testing.assert_allclose(M[e], Mt, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(b[e], bt, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(qdd[e], np.linalg.solve(Mt, -bt), rtol=1e-11, atol=1e-12)
    # the cart's position does not enter: a shifted cart has the same M and b
    q2 = q.clone()
    q2[:, 0] += 3.0
    assert torch.allclose(RO.mass_matrix(L, q2), torch.as_tensor(M), rtol=0, atol=1e-15)


def test_prismatic_tree_energy_and_power():
    """A random tree with about half its joints prismatic: M is the Hessian of
    the kinetic energy of differentiated kinematics, and the exact dynamics
    keep the power balance with contacts, damping and torques active."""
    wl = RS.tree_batch(seed=21, n_links=9, n_envs=3, prismatic=0.5, ground=0.0)
    L = wl.links
    kinds = [RO.prismatic(k) for k in L]
    assert 2 <= sum(kinds) <= 7, kinds
    q, qd = t64(wl.q0), t64(wl.qd0)
    M = RO.mass_matrix(L, q)
    for e in range(3):
        H = torch.autograd.functional.hessian(
            lambda v: _kinetic_from_motion(L, q[e:e + 1], v[None])[0], torch.zeros(len(L), dtype=DT64))
        assert torch.allclose(M[e], H, rtol=1e-10, atol=1e-14)
        assert torch.linalg.eigvalsh(M[e]).min() > 0
    prm = t64(wl.params)
    prm[:, 0] = 0.05
    pts = torch.stack([x[:, 2] for _, x in RO.contact_points(L, *RO.kinematics(L, q))], 1)
    prm[:, 4] = pts.median(1).values          # about half the contact spheres below the ground
    tau = t64(np.random.default_rng(22).standard_normal(q.shape))
    Qc = RO.contact_force(L, q, qd, prm)
    assert (Qc.abs().sum(1) > 0).all()
    qdd = RO.accel(L, q, qd, tau, prm, wl.gravity).detach()
    qa, qda = q.clone().requires_grad_(True), qd.clone().requires_grad_(True)
    En = (RO.kinetic(L, qa, qda) + RO.potential(L, qa, wl.gravity)).sum()
    gq, gqd = torch.autograd.grad(En, (qa, qda))
    dE = (gq * qd).sum(1) + (gqd * qdd).sum(1)
    power = (qd * (tau - prm[:, 0:1] * qd + Qc)).sum(1)
    assert torch.allclose(dE, power, rtol=1e-9, atol=1e-12)
