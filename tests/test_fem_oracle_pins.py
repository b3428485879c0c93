"""Pins of the FEM oracle (oracle/fem_oracle.py) to what the paper and the
mathematics fix, independently of the oracle's own formulas (CPU only).

Appendix D.2: linear tetrahedra, the stable neo-Hookean energy
Psi = mu/2 (I_C - 3) + lam/2 (J - alpha)^2 - mu/2 log(I_C + 1) integrated
over each element, forces from the energy gradient, semi-implicit Euler. The
activation, damping and ground readings are the oracle's (its header).
"""
import math

import numpy as np
import pytest
import torch
from scipy.optimize import brentq

from oracle import fem_oracle as FO
from paper_2412_12089_amd import fem_scenes as FS

DT64 = torch.float64


def psi_paper(F, mu, lam, a):
    """The energy of Appendix D.2 written out here from the formula (numpy),
    with the activation shifting the volume target."""
    Ic = float(np.sum(F * F))
    J = float(np.linalg.det(F))
    al = 1.0 + 3.0 * mu / (4.0 * lam)
    return 0.5 * mu * (Ic - 3.0) + 0.5 * lam * (J - al - a) ** 2 - 0.5 * mu * math.log(Ic + 1.0)


def total_energy(x, X, tets, mu, lam, a):
    """sum_e W_e Psi(D_s D_m^-1) assembled here in numpy."""
    E = 0.0
    for e, t in enumerate(tets):
        Dm = np.stack([X[t[1]] - X[t[0]], X[t[2]] - X[t[0]], X[t[3]] - X[t[0]]], axis=1)
        Ds = np.stack([x[t[1]] - x[t[0]], x[t[2]] - x[t[0]], x[t[3]] - x[t[0]]], axis=1)
        W = abs(np.linalg.det(Dm)) / 6.0
        E += W * psi_paper(Ds @ np.linalg.inv(Dm), mu, lam, a[e])
    return E


def piola(F, mu, lam, a=0.0, Fdot=None, damp=0.0):
    F = torch.as_tensor(F, dtype=DT64)
    Fd = torch.zeros_like(F) if Fdot is None else torch.as_tensor(Fdot, dtype=DT64)
    return FO.piola(F, Fd, torch.tensor(mu, dtype=DT64), torch.tensor(lam, dtype=DT64), damp,
                    torch.as_tensor(a, dtype=DT64)).numpy()


def rand_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


@pytest.mark.parametrize("scale", [0.05, 0.4])
def test_piola_is_the_gradient_of_the_papers_energy(scale):
    rng = np.random.default_rng(1)
    for _ in range(6):
        F = np.eye(3) + scale * rng.standard_normal((3, 3))
        mu, lam, a = rng.uniform(100, 2000), rng.uniform(100, 3000), rng.uniform(-0.3, 0.3)
        P = piola(F, mu, lam, a)
        h = 1e-6
        G = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                Fp, Fm = F.copy(), F.copy()
                Fp[i, j] += h
                Fm[i, j] -= h
                G[i, j] = (psi_paper(Fp, mu, lam, a) - psi_paper(Fm, mu, lam, a)) / (2 * h)
        assert np.allclose(P, G, rtol=1e-6, atol=1e-6 * np.abs(G).max())


def test_rest_shape_is_stress_free():
    rng = np.random.default_rng(2)
    for _ in range(5):
        P = piola(np.eye(3), rng.uniform(1, 5000), rng.uniform(1, 5000))
        assert np.abs(P).max() < 1e-10


def test_small_strain_limit_has_the_linearised_lame_pair():
    """F = I + eps (symmetric): P = 2 (3 mu / 4) eps + (lam - 5 mu / 8) tr(eps) I + O(eps^2)."""
    rng = np.random.default_rng(3)
    mu, lam = 1000.0, 1500.0
    A = rng.standard_normal((3, 3))
    eps = 1e-6 * (A + A.T)
    P = piola(np.eye(3) + eps, mu, lam)
    lin = 1.5 * mu * eps + (lam - 0.625 * mu) * np.trace(eps) * np.eye(3)
    assert np.abs(P - lin).max() < 1e-4 * np.abs(lin).max()


def test_stress_is_frame_indifferent():
    rng = np.random.default_rng(4)
    F = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    R = rand_rotation(rng)
    P, PR = piola(F, 800.0, 1200.0, 0.1), piola(R @ F, 800.0, 1200.0, 0.1)
    assert np.allclose(PR, R @ P, atol=1e-10 * np.abs(P).max())


def _two_cubes_state(seed=5):
    w = FS.two_cubes(seed=seed, n_envs=1)
    rng = np.random.default_rng(seed)
    X = w.X[0].astype(np.float64)
    x = X + 0.004 * rng.standard_normal(X.shape)
    a = rng.uniform(-0.2, 0.2, w.tets.shape[0])
    return w, X, x, a


def test_elastic_forces_are_minus_the_energy_gradient():
    w, X, x, a = _two_cubes_state()
    mu, lam = 900.0, 1300.0
    prm = torch.tensor([mu, lam, 1.0, 0.0, 0.0, 0.0, 0.0, -1e9], dtype=DT64)
    Bm, W, _ = FO.rest_data(X, w.tets)
    f = FO.elastic_forces(torch.tensor(x), torch.zeros(x.shape, dtype=DT64), w.tets, Bm, W, prm,
                          torch.tensor(a)).numpy()
    h = 1e-7
    g = np.zeros_like(x)
    for i in range(x.shape[0]):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            g[i, c] = (total_energy(xp, X, w.tets, mu, lam, a) - total_energy(xm, X, w.tets, mu, lam, a)) / (2 * h)
    assert np.allclose(f, -g, rtol=1e-5, atol=1e-6 * np.abs(g).max())


def test_internal_forces_conserve_momentum():
    w, X, x, a = _two_cubes_state(6)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(x.shape)
    Bm, W, _ = FO.rest_data(X, w.tets)
    # elasticity and activation: linear and angular momentum
    prm = torch.tensor([700.0, 900.0, 1.0, 0.0, 0.0, 0.0, 0.0, -1e9], dtype=DT64)
    f = FO.elastic_forces(torch.tensor(x), torch.tensor(v), w.tets, Bm, W, prm, torch.tensor(a)).numpy()
    scale = np.abs(f).max()
    assert np.abs(f.sum(0)).max() < 1e-11 * scale
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-11 * scale
    # the damping term is internal too: linear momentum
    prm[3] = 3.0
    fd = FO.elastic_forces(torch.tensor(x), torch.tensor(v), w.tets, Bm, W, prm, torch.tensor(a)).numpy()
    assert np.abs(fd.sum(0)).max() < 1e-11 * np.abs(fd).max()


def test_free_fall_of_the_rest_shape_is_exact():
    """At rest with no ground, every node falls as semi-implicit Euler of g:
    v_k = k dt g and x_k = x_0 + dt^2 g k (k + 1) / 2."""
    w = FS.two_cubes(n_envs=1)
    X = w.X[0].astype(np.float64)
    S, dt = 25, 2e-4
    prm = [1000.0, 1000.0, 1.0, 1.0, 100.0, 0.1, 0.1, -1.0]
    x, v = FO.rollout(FO.Mesh(w.tets), X, prm, X, np.zeros_like(X), np.zeros((S, w.tets.shape[0])), S, dt)
    g = np.array(FO.GRAVITY)
    assert np.allclose(v.numpy(), S * dt * g, atol=1e-12)
    assert np.allclose(x.numpy(), X + dt * dt * g * S * (S + 1) / 2, atol=1e-12)


def test_lumped_masses_hold_the_meshes_volume():
    h = 0.05
    Xm, tets = FS.cube_lattice_mesh([(0, 0, 0), (0, 0, 1)], h)
    _, W, wm = FO.rest_data(Xm, tets)
    assert abs(float(wm.sum()) - 2 * h ** 3) < 1e-18
    assert abs(float(W.sum()) - 2 * h ** 3) < 1e-18
    assert np.allclose(W.numpy(), h ** 3 / 6, rtol=1e-14)


@pytest.mark.parametrize("a", [0.25, -0.2])
def test_activation_sets_the_equilibrium_volume(a):
    """A lone element under activation a rests at uniform scale s* with
    d/ds Psi(s I) = 3 mu s - 3 mu s / (3 s^2 + 1) + 3 lam s^2 (s^3 - alpha - a) = 0:
    its forces vanish there, and a > 0 grows it."""
    mu, lam = 1000.0, 1000.0
    al = 1.0 + 0.75 * mu / lam

    def dpsi(s):
        return 3 * mu * s - 3 * mu * s / (3 * s * s + 1) + 3 * lam * s * s * (s ** 3 - al - a)

    s_star = brentq(dpsi, 0.5, 2.0, xtol=1e-15)
    assert (s_star > 1.0) == (a > 0)
    X = np.array([[0.0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [0, 0, 0.1]])
    tets = np.array([[0, 1, 2, 3]])
    Bm, W, _ = FO.rest_data(X, tets)
    prm = torch.tensor([mu, lam, 1.0, 0.0, 0.0, 0.0, 0.0, -1e9], dtype=DT64)
    zero = torch.zeros(4, 3, dtype=DT64)
    f_eq = FO.elastic_forces(torch.tensor(s_star * X), zero, tets, Bm, W, prm, torch.tensor([a])).numpy()
    f_rest = FO.elastic_forces(torch.tensor(X), zero, tets, Bm, W, prm, torch.tensor([a])).numpy()
    assert np.abs(f_eq).max() < 1e-7 * np.abs(f_rest).max()


def test_ground_contact_hand_values():
    """A rest element (no elastic force) with one node below the ground."""
    X = np.array([[0.0, 0, 0], [0.1, 0, 0.05], [0, 0.1, 0.05], [0, 0, 0.1]])
    tets = np.array([[0, 1, 2, 3]])
    x = X + np.array([0.3, 0.2, -0.004])   # node 0 at z = -0.004, the others above z = 0
    v = np.zeros((4, 3))
    v[:, :] = [0.5, -0.25, -1.5]            # rigid translation: no damping force
    ke, kd, kf = 300.0, 0.5, 0.2
    prm = torch.tensor([1000.0, 1000.0, 1.0, 2.0, ke, kd, kf, 0.0], dtype=DT64)
    Bm, W, _ = FO.rest_data(X, tets)
    f = (FO.elastic_forces(torch.tensor(x), torch.tensor(v), tets, Bm, W, prm, torch.zeros(1, dtype=DT64)) +
         FO.ground_forces(torch.tensor(x), torch.tensor(v), prm)).numpy()
    assert np.allclose(f[0], [-kf * 0.5, kf * 0.25, ke * 0.004 + kd * 1.5], atol=1e-9)
    assert np.abs(f[1:]).max() < 1e-9


def _case(seed=8, S=6):
    w = FS.two_cubes(seed=seed, n_envs=2, substeps=S)
    e = 0   # env 0 presses into the ground
    return FO.Mesh(w.tets), w.X[e], w.params[e], w.x0[e], w.v0[e], w.act[:, e], S, w.dt


def test_reverse_mode_matches_forward_mode():
    mesh, X, prm, x0, v0, act, S, dt = _case()
    rng = np.random.default_rng(9)
    gx, gv = rng.standard_normal(x0.shape), rng.standard_normal(x0.shape)
    t = (rng.standard_normal(x0.shape), rng.standard_normal(x0.shape), rng.standard_normal(act.shape),
         rng.standard_normal(8) * np.array([10, 10, 0.01, 0.1, 1, 0.01, 0.01, 0.001]))
    g = FO.rollout_vjp(mesh, X, prm, x0, v0, act, S, dt, gx, gv)
    tx, tv = FO.rollout_jvp(mesh, X, prm, x0, v0, act, S, dt, t)
    lhs = float((gx * tx.numpy()).sum() + (gv * tv.numpy()).sum())
    rhs = sum(float((gi.numpy() * ti).sum()) for gi, ti in zip(g, t))
    assert abs(lhs - rhs) < 1e-9 * max(abs(lhs), 1e-12)


def test_gradients_match_central_differences():
    mesh, X, prm, x0, v0, act, S, dt = _case(10)
    rng = np.random.default_rng(11)
    gx, gv = rng.standard_normal(x0.shape), 1e-3 * rng.standard_normal(x0.shape)
    gx0, gv0, gact, gprm = FO.rollout_vjp(mesh, X, prm, x0, v0, act, S, dt, gx, gv)

    def L(x0_, v0_, act_, prm_):
        x, v = FO.rollout(mesh, X, prm_, x0_, v0_, act_, S, dt)
        return float((x.numpy() * gx).sum() + (v.numpy() * gv).sum())

    x0 = x0.astype(np.float64); v0 = v0.astype(np.float64); act = act.astype(np.float64)
    prm = np.asarray(prm, dtype=np.float64)
    for name, base, grad, h in (("x0", x0, gx0, 1e-6), ("v0", v0, gv0, 1e-4), ("act", act, gact, 1e-5),
                                ("prm", prm, gprm, None)):
        d = rng.standard_normal(base.shape)
        if name == "prm":
            d = d * prm * 1e-6
            d[7] = 1e-7   # ground height
            h = 1.0
        args = {"x0": x0, "v0": v0, "act": act, "prm": prm}
        ap, am = dict(args), dict(args)
        ap[name] = base + h * d
        am[name] = base - h * d
        fd = (L(**{k + "_": v for k, v in ap.items()}) - L(**{k + "_": v for k, v in am.items()})) / (2 * h)
        an = float((grad.numpy() * d).sum())
        assert abs(fd - an) < 1e-5 * max(abs(an), 1e-12), (name, fd, an)


def test_rho_cotangent_follows_the_scale_identity():
    """Scaling mu, lam, rho, damp, k_e, k_d, k_f together leaves f / m unchanged."""
    mesh, X, prm, x0, v0, act, S, dt = _case(12)
    rng = np.random.default_rng(13)
    g = FO.rollout_vjp(mesh, X, prm, x0, v0, act, S, dt, rng.standard_normal(x0.shape),
                       rng.standard_normal(x0.shape))[3].numpy()
    p = np.asarray(prm)
    scaled = sum(p[i] * g[i] for i in (0, 1, 3, 4, 5, 6))
    assert abs(p[2] * g[2] + scaled) < 1e-9 * max(abs(scaled), 1e-12)
