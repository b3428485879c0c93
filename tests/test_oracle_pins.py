"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, an invariant of the
transfer, a library routine (scipy/numpy), an energy derivative taken by a
different route, exact rational arithmetic, or finite differences.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import mpm_oracle as O

DT = torch.float64


def rand_rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def blob(rng, N, lo, hi):
    return torch.from_numpy(rng.uniform(lo, hi, size=(N, 3)).astype(np.float32)).to(DT)


def params(E=5e3, nu=0.3, rho=1e3, Vp=1e-6, sy=50.0, K=1e4, gamma=7.0):
    return torch.tensor([E, nu, rho, Vp, sy, K, gamma], dtype=DT)


# ---------------------------------------------------------------- Lame parameters
def test_lame_textbook_values():
    # E = 1, nu = 1/4 gives mu = lam = 2/5; nu = 0 gives lam = 0 and mu = E/2
    mu, lam = O.lame(1.0, 0.25)
    assert abs(mu - 0.4) < 1e-15 and abs(lam - 0.4) < 1e-15
    mu, lam = O.lame(7.0, 0.0)
    assert lam == 0.0 and abs(mu - 3.5) < 1e-15


@pytest.mark.parametrize("E,nu", [(5e3, 0.3), (1e4, 0.25), (4e3, 0.2), (2.0, -0.4), (1.0, 0.49)])
def test_lame_reproduces_the_elastic_moduli(E, nu):
    # the defining experiments of E and nu on the isotropic linear law s = lam tr(e) I + 2 mu e:
    # a uniaxial strain state e = diag(1, -nu, -nu) carries stress E along x and none across;
    # a uniform dilation carries 3 K per unit strain, K = E / (3 (1 - 2 nu)); pure shear carries 2 G
    mu, lam = O.lame(E, nu)
    lin = lambda e: lam * np.trace(e) * np.eye(3) + 2.0 * mu * e
    s = lin(np.diag([1.0, -nu, -nu]))
    np.testing.assert_allclose(np.diag(s), [E, 0.0, 0.0], atol=1e-12 * E)
    np.testing.assert_allclose(lin(np.eye(3)), 3.0 * E / (3.0 * (1.0 - 2.0 * nu)) * np.eye(3), rtol=1e-13)
    shear = np.zeros((3, 3)); shear[0, 1] = shear[1, 0] = 1.0
    np.testing.assert_allclose(lin(shear)[0, 1], 2.0 * E / (2.0 * (1.0 + nu)), rtol=1e-13)


@pytest.mark.parametrize("mat", [O.COROTATED, O.VONMISES])
def test_small_strain_stress_is_the_linear_law(mat):
    # corotated and Hencky elasticity linearise at F = I to the isotropic law with the Lame pair of
    # (E, nu): a uniaxial stretch with lateral contraction nu carries tau_xx = E eps, no lateral stress
    E, nu, eps = 5e3, 0.3, 1e-7
    mu, lam = O.lame(torch.tensor(E, dtype=DT), torch.tensor(nu, dtype=DT))
    F = torch.diag(torch.tensor([1.0 + eps, 1.0 - nu * eps, 1.0 - nu * eps], dtype=DT))[None]
    tau = O.stress(mat, F, mu, lam, torch.tensor(1e4, dtype=DT), torch.tensor(7.0, dtype=DT))[0].numpy()
    np.testing.assert_allclose(tau[0, 0] / eps, E, rtol=1e-5)
    assert abs(tau[1, 1]) < 1e-5 * E * eps and abs(tau[2, 2]) < 1e-5 * E * eps
    assert np.abs(tau - np.diag(np.diag(tau))).max() < 1e-9 * E * eps


def test_stable_neohookean_small_strain_closed_form():
    # the stable neo-Hookean energy written in the Lame pair (mu, lam) linearises at F = I to
    # 2 (3 mu / 4) e + (lam - 5 mu / 8) tr(e) I: derivative of mu (1 - 1/(I_C + 1)) F at I_C = 3 is
    # (3 mu / 4) e + (mu / 8) tr(e) I, and of lam (J - alpha) J F^-T with alpha = 1 + 3 mu / (4 lam)
    # is lam tr(e) I - (3 mu / 4)(tr(e) I - e^T); summed for a symmetric strain e
    rng = np.random.default_rng(3)
    mu, lam = 1234.0, 2345.0
    e = 1e-7 * rng.standard_normal((3, 3))
    e = 0.5 * (e + e.T)
    F = torch.from_numpy(np.eye(3) + e)[None]
    tau = O.stress(O.NEOHOOKEAN, F, torch.tensor(mu, dtype=DT), torch.tensor(lam, dtype=DT),
                   torch.tensor(0.0, dtype=DT), torch.tensor(1.0, dtype=DT))[0].numpy()
    lin = 2.0 * (0.75 * mu) * e + (lam - 0.625 * mu) * np.trace(e) * np.eye(3)
    np.testing.assert_allclose(tau, lin, atol=1e-5 * np.abs(lin).max())


# ---------------------------------------------------------------- weights
def test_bspline_closed_form_values():
    # quadratic B-spline at f = 1 (particle on a cell centre) and f = 1/2 (on a node)
    x = torch.tensor([[1.0 / 32, 1.0 / 32, 1.0 / 32], [0.5 / 32, 0.5 / 32, 0.5 / 32]], dtype=DT)
    base, W, d, _ = O.stencil(x, 32)
    w1 = np.array([1 / 8, 3 / 4, 1 / 8])
    w05 = np.array([1 / 2, 1 / 2, 0.0])
    assert base[0].tolist() == [0, 0, 0] and base[1].tolist() == [0, 0, 0]
    np.testing.assert_allclose(W[0].numpy(), np.einsum("a,b,c->abc", w1, w1, w1).reshape(-1), atol=1e-15)
    np.testing.assert_allclose(W[1].numpy(), np.einsum("a,b,c->abc", w05, w05, w05).reshape(-1), atol=1e-15)


def test_bspline_partition_of_unity_and_linear_reproduction():
    rng = np.random.default_rng(0)
    x = blob(rng, 500, 0.2, 0.8)
    _, W, d, _ = O.stencil(x, 48)
    np.testing.assert_allclose(W.sum(1).numpy(), 1.0, atol=1e-14)
    np.testing.assert_allclose((W[..., None] * d).sum(1).numpy(), 0.0, atol=1e-16)
    # second moment of the quadratic B-spline: sum w d d^T = dx^2/4 I
    D = torch.einsum("pk,pki,pkj->pij", W, d, d)
    np.testing.assert_allclose(D.numpy(), np.broadcast_to(np.eye(3) / (4 * 48 ** 2), D.shape), atol=1e-16)


# ---------------------------------------------------------------- keys
def test_base_cells_exact_at_boundaries():
    n = 48
    xs = []
    for k in range(0, n - 2):
        x0 = np.float32((k + 0.5) / n)
        xs += [x0, np.nextafter(x0, np.float32(0)), np.nextafter(x0, np.float32(1))]
    xs = np.array(xs, dtype=np.float32)
    a = O.base_cells(xs, n)
    b = O.base_cells_exact(xs, n)
    assert (a == b).all()


def test_cell_keys_bruteforce_and_stable_perm():
    rng = np.random.default_rng(1)
    n = 32
    x = rng.uniform(0.1, 0.9, size=(300, 3)).astype(np.float32)
    x[10] = x[11]  # a duplicate key: the stable order keeps 10 before 11
    keys = O.cell_keys(x, n)
    for p in range(len(x)):
        b = [min(max(int(O.base_cells_exact(x[p:p + 1, a], n)[0]), 0), n - 3) for a in range(3)]
        T = n // 4
        tile = ((b[0] // 4) * T + b[1] // 4) * T + b[2] // 4
        cell = ((b[0] % 4) * 4 + b[1] % 4) * 4 + b[2] % 4
        assert keys[p] == tile * 64 + cell
    perm = O.sort_permutation(keys)
    sk = keys[perm]
    assert (np.diff(sk) >= 0).all()
    for j in range(len(perm) - 1):
        if sk[j] == sk[j + 1]:
            assert perm[j] < perm[j + 1]


# ---------------------------------------------------------------- matrix functions vs library
def test_matrix_functions_match_scipy():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((20, 3, 3))
    spd = A @ A.transpose(0, 2, 1) + 0.3 * np.eye(3)
    near_i = np.eye(3) + 0.05 * (A + A.transpose(0, 2, 1))
    rots = [rand_rot(rng) for _ in range(5)]
    rep = np.stack([R @ np.diag([1.2, 1.2, 0.7]) @ R.T for R in rots])   # a repeated eigenvalue
    for Bs in (spd, near_i, rep):
        Bt = torch.from_numpy(Bs)
        L = O.logm_spd(Bt).numpy()
        S = O.sqrtm_spd(Bt).numpy()
        for i in range(len(Bs)):
            np.testing.assert_allclose(L[i], scipy.linalg.logm(Bs[i]).real, atol=1e-11)
            np.testing.assert_allclose(S[i], scipy.linalg.sqrtm(Bs[i]).real, atol=1e-11)
    X = 0.7 * (A + A.transpose(0, 2, 1))
    Ex = O.expm_sym(torch.from_numpy(X)).numpy()
    for i in range(len(X)):
        np.testing.assert_allclose(Ex[i], scipy.linalg.expm(X[i]), rtol=1e-12, atol=1e-12)
    F = np.eye(3) + 0.4 * A
    F = F[np.linalg.det(F) > 0.05]
    R = O.polar_rotation(torch.from_numpy(F)).numpy()
    for i in range(len(F)):
        u, _ = scipy.linalg.polar(F[i])
        np.testing.assert_allclose(R[i], u, atol=1e-12)


# ---------------------------------------------------------------- constitutive
ENERGY_MATS = [O.NEOHOOKEAN, O.COROTATED, O.VONMISES, O.FLUID_TAIT, O.FLUID_PAPER]


def energy_density(mat, F, mu, lam, K, gamma):
    """Strain-energy densities, written from singular values (a different route from the oracle)."""
    J = torch.linalg.det(F)
    if mat == O.NEOHOOKEAN:
        Ic = (F * F).sum((-1, -2))
        alpha = 1 + 3 * mu / (4 * lam)
        return mu / 2 * (Ic - 3) + lam / 2 * (J - alpha) ** 2 - mu / 2 * torch.log(Ic + 1)
    s = torch.linalg.svdvals(F)
    if mat == O.COROTATED:
        return mu * ((s - 1) ** 2).sum(-1) + lam / 2 * (J - 1) ** 2
    if mat == O.VONMISES:
        e = torch.log(s)
        return mu * (e ** 2).sum(-1) + lam / 2 * e.sum(-1) ** 2
    if mat == O.FLUID_TAIT:
        # pressure p = K (J^-gamma - 1) = -dPsi/dJ
        return -K * (J ** (1 - gamma) / (1 - gamma) - J)
    if mat == O.FLUID_PAPER:
        return lam / 2 * (J - 1) ** 2
    raise ValueError


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_stress_is_energy_derivative(mat):
    rng = np.random.default_rng(3 + mat)
    A = rng.standard_normal((16, 3, 3))
    F = torch.from_numpy(np.eye(3) + 0.15 * A).requires_grad_(True)
    mu, lam = O.lame(torch.tensor(5e3, dtype=DT), torch.tensor(0.3, dtype=DT))
    K, gam = torch.tensor(1e4, dtype=DT), torch.tensor(7.0, dtype=DT)
    psi = energy_density(mat, F, mu, lam, K, gam).sum()
    (P,) = torch.autograd.grad(psi, F)
    tau_ref = P @ F.detach().transpose(-1, -2)
    tau = O.stress(mat, F.detach(), mu, lam, K, gam)
    np.testing.assert_allclose(tau.numpy(), tau_ref.numpy(), rtol=1e-9, atol=1e-8 * 5e3)
    np.testing.assert_allclose(tau.numpy(), tau.transpose(-1, -2).numpy(), atol=1e-9 * 5e3)


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_stress_vanishes_at_rest_and_under_rotation(mat):
    rng = np.random.default_rng(7)
    mu, lam = O.lame(torch.tensor(5e3, dtype=DT), torch.tensor(0.3, dtype=DT))
    K, gam = torch.tensor(1e4, dtype=DT), torch.tensor(7.0, dtype=DT)
    F = torch.from_numpy(np.stack([np.eye(3)] + [rand_rot(rng) for _ in range(6)]))
    tau = O.stress(mat, F, mu, lam, K, gam)
    assert tau.abs().max().item() < 1e-9


def test_fluid_stress_depends_only_on_J():
    rng = np.random.default_rng(8)
    F = torch.from_numpy(np.eye(3) + 0.2 * rng.standard_normal((10, 3, 3)))
    J = torch.linalg.det(F)
    Fi = (J ** (1 / 3))[:, None, None] * torch.eye(3, dtype=DT)
    mu, lam = O.lame(torch.tensor(5e3, dtype=DT), torch.tensor(0.3, dtype=DT))
    for mat in (O.FLUID_TAIT, O.FLUID_PAPER):
        a = O.stress(mat, F, mu, lam, torch.tensor(1e4, dtype=DT), torch.tensor(7.0, dtype=DT))
        b = O.stress(mat, Fi, mu, lam, torch.tensor(1e4, dtype=DT), torch.tensor(7.0, dtype=DT))
        np.testing.assert_allclose(a.numpy(), b.numpy(), rtol=1e-12, atol=1e-9)


# ---------------------------------------------------------------- return mapping
def test_von_mises_return_closed_form():
    rng = np.random.default_rng(9)
    mu, lam = O.lame(torch.tensor(5e3, dtype=DT), torch.tensor(0.2, dtype=DT))
    sy = torch.tensor(50.0, dtype=DT)
    Y = O.YIELD_SCALE * 50.0 / (2 * mu.item())
    for trial in range(40):
        s = np.exp(rng.uniform(-0.08, 0.08, size=3))
        R1, R2 = rand_rot(rng), rand_rot(rng)
        F = torch.from_numpy((R1 @ np.diag(s) @ R2)[None])
        Fp = O.project(O.VONMISES, F, mu, sy)[0].numpy()
        e = np.log(s)
        eh = e - e.mean()
        nrm = np.linalg.norm(eh)
        if nrm - Y > 0:
            e_new = e.mean() + eh * (Y / nrm)      # on the yield surface, same trace
            expect = R1 @ np.diag(np.exp(e_new)) @ R2
            assert abs(np.linalg.norm(e_new - e_new.mean()) - Y) < 1e-12
            assert abs(e_new.sum() - e.sum()) < 1e-12
        else:
            expect = F[0].numpy()                  # inside the yield surface: elastic
        np.testing.assert_allclose(Fp, expect, atol=1e-12)


def test_fluid_projection_keeps_volume():
    rng = np.random.default_rng(10)
    F = torch.from_numpy(np.eye(3) + 0.1 * rng.standard_normal((20, 3, 3)))
    for mat in (O.FLUID_TAIT, O.FLUID_PAPER):
        Fp = O.project(mat, F, torch.tensor(1.0, dtype=DT), torch.tensor(0.0, dtype=DT))
        np.testing.assert_allclose(torch.linalg.det(Fp).numpy(), torch.linalg.det(F).numpy(), rtol=1e-13)
        off = Fp - Fp.diagonal(dim1=-2, dim2=-1).mean(-1)[:, None, None] * torch.eye(3, dtype=DT)
        assert off.abs().max().item() < 1e-15


# ---------------------------------------------------------------- transfer invariants
def scene(mat, N=400, n=32, lo=0.35, hi=0.6, seed=11, v_scale=0.5, F_scale=0.0, C_scale=0.0):
    rng = np.random.default_rng(seed)
    x = blob(rng, N, lo, hi)
    v = torch.from_numpy(rng.uniform(-v_scale, v_scale, size=(N, 3))).to(DT)
    C = torch.from_numpy(C_scale * rng.standard_normal((N, 3, 3)))
    F = torch.from_numpy(np.eye(3) + F_scale * rng.standard_normal((N, 3, 3)))
    env = O.Env(n=n, dt=1e-4, material=mat, gravity=(0.0, 0.0, 0.0))
    return env, (x, v, C, F)


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_p2g_mass_exact_and_momentum_conserved(mat):
    env, (x, v, C, F) = scene(mat, F_scale=0.05, C_scale=3.0)
    prm = params(Vp=1e-5)
    gm, gP, _ = O.p2g(env, prm, x, v, C, F)
    mp = prm[2] * prm[3]
    assert abs(gm.sum().item() - mp.item() * len(x)) <= 1e-14 * mp.item() * len(x)
    # APIC and the stress impulse carry no net momentum: sum_i w d = 0
    np.testing.assert_allclose(gP.sum(0).numpy(), (mp * v).sum(0).numpy(), rtol=0, atol=1e-13)
    gv = O.grid_update(env, gm, gP, 0.0)
    xn, vn, Cn, Fn = O.g2p(env, prm, x, F, gv)
    # G2P conserves momentum: sum_p m_p v_p' = sum_i m_i v_i
    np.testing.assert_allclose((mp * vn).sum(0).numpy(), (gm[:, None] * gv).sum(0).numpy(), atol=1e-13)


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_free_fall_closed_form(mat):
    rng = np.random.default_rng(12)
    N, n, S, dt = 300, 32, 12, 1e-4
    x0 = blob(rng, N, 0.4, 0.6)
    v0 = torch.tensor([0.3, -0.2, 0.1], dtype=DT)
    g = torch.tensor([0.0, 0.0, -9.8], dtype=DT)
    state = (x0, v0.expand(N, 3).clone(), torch.zeros(N, 3, 3, dtype=DT),
             torch.eye(3, dtype=DT).expand(N, 3, 3).clone())
    env = O.Env(n=n, dt=dt, material=mat, gravity=tuple(g.tolist()))
    (x, v, C, F), oob = O.rollout(env, params(Vp=1e-6), state, S)
    assert not oob
    np.testing.assert_allclose(v.numpy(), (v0 + S * dt * g).expand(N, 3).numpy(), atol=1e-12)
    np.testing.assert_allclose(x.numpy(), (x0 + S * dt * v0 + dt * dt * g * S * (S + 1) / 2).numpy(), atol=1e-13)
    assert C.abs().max().item() < 1e-9
    np.testing.assert_allclose(F.numpy(), np.broadcast_to(np.eye(3), F.shape), atol=1e-12)


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_rest_state_stays_at_rest(mat):
    rng = np.random.default_rng(13)
    N = 300
    x0 = blob(rng, N, 0.4, 0.6)
    state = (x0, torch.zeros(N, 3, dtype=DT), torch.zeros(N, 3, 3, dtype=DT),
             torch.eye(3, dtype=DT).expand(N, 3, 3).clone())
    env = O.Env(n=32, dt=1e-4, material=mat, gravity=(0.0, 0.0, 0.0))
    (x, v, C, F), _ = O.rollout(env, params(Vp=1e-6), state, 5)
    assert (x - x0).abs().max().item() < 1e-15
    assert v.abs().max().item() < 1e-12


def test_affine_velocity_field_is_reproduced():
    # APIC reproduces v = v0 + B x exactly (tau = 0 with a zero-stiffness corotated body)
    rng = np.random.default_rng(14)
    N, n, dt = 400, 32, 1e-3
    x = blob(rng, N, 0.35, 0.6)
    B = torch.from_numpy(rng.standard_normal((3, 3)))
    v0 = torch.tensor([0.1, 0.2, -0.3], dtype=DT)
    v = v0 + x @ B.T
    F0 = torch.from_numpy(np.eye(3) + 0.1 * rng.standard_normal((N, 3, 3)))
    env = O.Env(n=n, dt=dt, material=O.COROTATED, gravity=(0.0, 0.0, 0.0))
    prm = params(E=0.0, nu=0.3, Vp=1e-6)
    xn, vn, Cn, Fn, _ = O.substep(env, prm, x, v, B.expand(N, 3, 3).clone(), F0, 0.0)
    np.testing.assert_allclose(vn.numpy(), v.numpy(), atol=1e-12)
    np.testing.assert_allclose(Cn.numpy(), B.expand(N, 3, 3).numpy(), atol=1e-10)
    np.testing.assert_allclose(xn.numpy(), (x + dt * v).numpy(), atol=1e-14)
    np.testing.assert_allclose(Fn.numpy(), ((torch.eye(3, dtype=DT) + dt * B) @ F0).numpy(), atol=1e-12)


@pytest.mark.parametrize("mat", ENERGY_MATS)
def test_grid_force_is_minus_energy_gradient(mat):
    # the MLS-MPM stress impulse equals -dt dE/du_i, E = sum_p Vp Psi((I + sum_i 4 n^2 w u_i d^T) F)
    rng = np.random.default_rng(15 + mat)
    N, n, dt, Vp = 200, 32, 1e-4, 2e-6
    x = blob(rng, N, 0.4, 0.55)
    F = torch.from_numpy(np.eye(3) + 0.08 * rng.standard_normal((N, 3, 3)))
    prm = params(Vp=Vp)
    env = O.Env(n=n, dt=dt, material=mat, gravity=(0.0, 0.0, 0.0))
    zeros3 = torch.zeros(N, 3, dtype=DT)
    gm, gP, _ = O.p2g(env, prm, x, zeros3, torch.zeros(N, 3, 3, dtype=DT), F)
    base, W, d, _ = O.stencil(x, n)
    lin = O.node_index(base, n)
    u = torch.zeros(n ** 3, 3, dtype=DT, requires_grad=True)
    ui = u[lin]                                                 # [N,27,3]
    Fhat = (torch.eye(3, dtype=DT) + 4 * n * n * torch.einsum("pk,pki,pkj->pij", W, ui, d)) @ F
    mu, lam = O.lame(prm[0], prm[1])
    energy = Vp * energy_density(mat, Fhat, mu, lam, prm[5], prm[6]).sum()
    (gE,) = torch.autograd.grad(energy, u)
    np.testing.assert_allclose(gP.numpy(), (-dt * gE).numpy(), rtol=1e-9, atol=1e-9 * gP.abs().max().item())


# ---------------------------------------------------------------- grid boundary pieces
def test_walls_zero_the_boundary_layer():
    n, b = 16, 3
    wm = O.wall_mask(n, b).reshape(n, n, n)
    assert wm[:b].all() and wm[n - b:].all() and wm[:, :b].all() and wm[:, :, n - b:].all()
    assert not wm[b:n - b, b:n - b, b:n - b].any()
    assert int(wm.sum()) == n ** 3 - (n - 2 * b) ** 3


def test_contact_projection_hand_values():
    # one node deep inside a static box (s = 1) moving against the +x face's normal
    n = 16
    box = O.Box(center=(0.5, 0.5, 0.5), half=(0.2, 0.2, 0.2), velocity=(0.0, 0.0, 0.0), alpha=32.0, mu_b=0.5)
    env = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=box)
    pos = O.node_positions(n)
    i_in = int(((pos - torch.tensor([0.6875, 0.5, 0.5], dtype=DT)).abs().sum(1)).argmin())  # d = -0.0125, normal +x
    v = torch.zeros(n ** 3, 3, dtype=DT)
    act = torch.ones(n ** 3, dtype=torch.bool)
    cases = [((-1.0, 0.2, 0.0), (0.0, 0.0, 0.0)),        # |u_t| = 0.2 <= 0.5: sticks
             ((-1.0, 2.0, 0.0), (0.0, 1.5, 0.0)),        # slides: u_t (1 - 0.5 * 1 / 2)
             ((1.0, 2.0, 0.0), (1.0, 2.0, 0.0))]         # separating: unchanged
    for vin, vout in cases:
        v[i_in] = torch.tensor(vin, dtype=DT)
        out = O.collide(env, v, *O.collider_motion(env, 0.0)[:2], act)
        np.testing.assert_allclose(out[i_in].numpy(), vout, atol=1e-14)
    # a node outside at distance d: blend s = exp(-alpha d) of projected and free velocity
    i_out = int(((pos - torch.tensor([0.75, 0.5, 0.5], dtype=DT)).abs().sum(1)).argmin())  # d = 0.05
    v[i_out] = torch.tensor([-1.0, 0.2, 0.0], dtype=DT)
    out = O.collide(env, v, *O.collider_motion(env, 0.0)[:2], act)
    s = math.exp(-32.0 * 0.05)
    np.testing.assert_allclose(out[i_out].numpy(), [(1 - s) * -1.0, (1 - s) * 0.2, 0.0], atol=1e-14)


def test_box_sdf_face_edge_corner_hand_values():
    # box centred at c with half extents (0.2, 0.1, 0.15); points placed by hand outside a face,
    # an edge and a corner, and inside near a face, with the distance and outward normal worked out
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    h = torch.tensor([0.2, 0.1, 0.15], dtype=DT)
    cases = [
        # (offset from c, distance, normal)
        ((0.0, 0.0, -0.2), 0.05, (0.0, 0.0, -1.0)),                    # below the -z face
        ((0.23, 0.14, 0.0), 0.05, (0.6, 0.8, 0.0)),                    # outside the (+x, +y) edge: 3-4-5
        ((-0.23, 0.0, 0.19), 0.05, (-0.6, 0.0, 0.8)),                  # outside the (-x, +z) edge
        ((0.22, -0.13, 0.21), 0.07, (2 / 7, -3 / 7, 6 / 7)),           # outside a corner: 2-3-6-7
        ((0.19, 0.08, 0.0), -0.01, (1.0, 0.0, 0.0)),                   # inside, nearest the +x face
        ((0.05, -0.09, 0.1), -0.01, (0.0, -1.0, 0.0)),                 # inside, nearest the -y face
    ]
    p = c + torch.tensor([o for o, _, _ in cases], dtype=DT)
    d, nrm = O.box_sdf(p, c, h)
    np.testing.assert_allclose(d.numpy(), [dd for _, dd, _ in cases], atol=1e-14)
    np.testing.assert_allclose(nrm.numpy(), [nn for _, _, nn in cases], atol=1e-13)
    # exact ties inside (dyadic numbers, so |rel| - half ties exactly): the first tied axis wins
    h2 = torch.tensor([0.25, 0.125, 0.375], dtype=DT)
    ties = [((-0.1875, 0.0625, -0.3125), (-1.0, 0.0, 0.0)),    # x, y and z tie at -1/16
            ((0.0, -0.0625, 0.3125), (0.0, -1.0, 0.0))]       # y and z tie at -1/16
    p2 = c + torch.tensor([o for o, _ in ties], dtype=DT)
    d2, n2 = O.box_sdf(p2, c, h2)
    np.testing.assert_allclose(d2.numpy(), [-0.0625, -0.0625], atol=0)
    np.testing.assert_allclose(n2.numpy(), [nn for _, nn in ties], atol=0)
    # the normal is the gradient of the distance wherever the distance is differentiable
    pg = p[:6].clone().requires_grad_(True)
    dg, _ = O.box_sdf(pg, c, h)
    (g,) = torch.autograd.grad(dg.sum(), pg)
    np.testing.assert_allclose(g.numpy(), nrm[:6].numpy(), atol=1e-13)


# ---------------------------------------------------------------- gradients
def tiny(mat, collider=False, seed=20, N=48):
    rng = np.random.default_rng(seed)
    n = 16
    x = blob(rng, N, 0.36, 0.55)
    v = torch.from_numpy(rng.uniform(-0.5, 0.5, size=(N, 3)))
    C = torch.from_numpy(2.0 * rng.standard_normal((N, 3, 3)))
    Fs = np.full((N, 1, 1), 0.05)
    if mat == O.VONMISES:
        Fs[::2] = 0.12      # half the particles start beyond the yield surface, half well inside
        Fs[1::2] = 0.002
    F = torch.from_numpy(np.eye(3) + Fs * rng.standard_normal((N, 3, 3)))
    if mat in (O.FLUID_TAIT, O.FLUID_PAPER):
        F = (torch.linalg.det(F) ** (1 / 3))[:, None, None] * torch.eye(3, dtype=DT)
    box = None
    if collider:
        box = O.Box(center=(0.62, 0.45, 0.45), half=(0.05, 0.2, 0.2), velocity=(-0.3, 0.0, 0.0),
                    alpha=2.0 * n, mu_b=0.5)
    env = O.Env(n=n, dt=2e-4, material=mat, collider=box)
    prm = params(E=5e3, nu=0.3, Vp=(0.19 ** 3) / N, sy=30.0)
    return env, prm, (x, v, C, F)


GRAD_CASES = [(m, False) for m in ENERGY_MATS] + [(O.FLUID_TAIT, True)]


@pytest.mark.parametrize("mat,collider", GRAD_CASES)
def test_reverse_mode_matches_forward_mode(mat, collider):
    env, prm, st = tiny(mat, collider)
    S = 3
    rng = np.random.default_rng(30)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp = O.rollout_vjp(env, prm, st, S, cot)
    for _ in range(4):
        tan = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
        tp = torch.from_numpy(rng.standard_normal(7)) * prm.abs() * 1e-3
        out = O.rollout_jvp(env, prm, st, S, tan, tp)
        lhs = sum((a * b).sum() for a, b in zip(out, cot)).item()
        rhs = (sum((a * b).sum() for a, b in zip(tan, g)) + (gp * tp).sum()).item()
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs))


def _loss(env, prm, st, S, cot):
    (x, v, C, F), _ = O.rollout(env, prm, st, S)
    return sum((a * b).sum() for a, b in zip((x, v, C, F), cot)).item()


@pytest.mark.parametrize("mat,collider", GRAD_CASES)
def test_reverse_mode_matches_central_differences(mat, collider):
    env, prm, st = tiny(mat, collider)
    S = 3
    rng = np.random.default_rng(31)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp = O.rollout_vjp(env, prm, st, S, cot)
    # random directions in state space and along E (and sigma_y for von Mises)
    for trial in range(3):
        tan = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
        if mat in (O.FLUID_TAIT, O.FLUID_PAPER):
            tan[3] = torch.zeros_like(tan[3])
        scale = [1e-6, 1e-6, 1e-6, 1e-6]
        h = [s * t for s, t in zip(scale, tan)]
        plus = [a + b for a, b in zip(st, h)]
        minus = [a - b for a, b in zip(st, h)]
        fd = (_loss(env, prm, plus, S, cot) - _loss(env, prm, minus, S, cot)) / 2
        an = sum((a * b).sum() for a, b in zip(h, g)).item()
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * sum(abs(x) for x in (fd, an)) + 1e-12), (fd, an)
    for k in (0, 1, 4, 5, 6):
        if prm[k] == 0:
            continue
        hk = 1e-6 * prm[k].item()
        pp, pm = prm.clone(), prm.clone()
        pp[k] += hk
        pm[k] -= hk
        fd = (_loss(env, pp, st, S, cot) - _loss(env, pm, st, S, cot)) / (2 * hk)
        an = gp[k].item()
        assert abs(fd - an) <= 1e-5 * max(abs(an), abs(fd)) + 1e-9, (k, fd, an)


@pytest.mark.parametrize("mat,collider", GRAD_CASES)
def test_density_and_volume_cotangents(mat, collider):
    # with one particle mass m_p = rho Vp per environment, the grid velocity P_i / m_i depends on the
    # particle volume only through tau / rho (Vp cancels) and the yield offset through sigma_y / E.
    # So the loss is unchanged when (rho, E, sigma_y, K) are scaled together, and does not depend on
    # Vp at all: rho dL/drho = -(E dL/dE + sigma_y dL/dsigma_y + K dL/dK) and dL/dVp = 0. Central
    # differences in rho and Vp check the same two numbers directly.
    env, prm, st = tiny(mat, collider)
    S = 3
    rng = np.random.default_rng(32)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    _, gp = O.rollout_vjp(env, prm, st, S, cot)
    g = gp.numpy()
    p = prm.numpy()
    euler = p[0] * g[0] + p[4] * g[4] + p[5] * g[5]
    scale = abs(p[0] * g[0]) + abs(p[4] * g[4]) + abs(p[5] * g[5])
    assert scale > 0
    assert abs(p[2] * g[2] + euler) <= 1e-9 * scale, (p[2] * g[2], euler)
    assert abs(p[3] * g[3]) <= 1e-9 * scale
    for k in (2, 3):
        hk = 1e-6 * prm[k].item()
        pp, pm = prm.clone(), prm.clone()
        pp[k] += hk
        pm[k] -= hk
        fd = (_loss(env, pp, st, S, cot) - _loss(env, pm, st, S, cot)) / (2 * hk)
        assert abs(fd * p[k] - g[k] * p[k]) <= 1e-6 * scale, (k, fd, g[k])


def test_von_mises_tiny_scene_is_plastic():
    # the gradient cases above must exercise the return mapping, not only the elastic branch
    env, prm, (x, v, C, F) = tiny(O.VONMISES)
    mu, _ = O.lame(prm[0], prm[1])
    Fp = O.project(O.VONMISES, F, mu, prm[4])
    moved = ((Fp - F).flatten(1).norm(dim=1) > 1e-12).sum().item()
    assert 0 < moved < len(F)


# ---------------------------------------------------------------- prescribed collider motion (actions)
def _moving_box(S, seed, edge=False):
    import dataclasses
    env, prm, st = tiny(O.FLUID_TAIT, collider=True)
    if edge:   # the blob meets the box along an edge, where the normal turns with the center
        env = dataclasses.replace(env, collider=dataclasses.replace(env.collider, center=(0.6, 0.6, 0.45),
                                                                    half=(0.05, 0.06, 0.2), mu_b=0.3))
    rng = np.random.default_rng(seed)
    vb = torch.tensor(env.collider.velocity, dtype=DT)
    vel = vb + 0.2 * torch.from_numpy(rng.standard_normal((S, 3)))
    return env, prm, st, vel


def test_constant_actions_reproduce_the_fixed_velocity_box():
    # a box driven by per-substep velocities all equal to v_b follows c0 + t v_b
    env, prm, st = tiny(O.FLUID_TAIT, collider=True)
    S = 4
    vel = torch.tensor(env.collider.velocity, dtype=DT).expand(S, 3).clone()
    a, _ = O.rollout(env, prm, st, S)
    b, _ = O.rollout(env, prm, st, S, vel=vel)
    for u, w in zip(a, b):
        np.testing.assert_allclose(u.numpy(), w.numpy(), rtol=0, atol=1e-12)
    path = O.collider_path(env, vel)
    for k in range(S):
        np.testing.assert_allclose(path[k].numpy(), np.array(env.collider.center) + k * env.dt * vel[0].numpy(),
                                   rtol=0, atol=1e-15)


def test_moving_box_actually_pushes():
    # the box is in contact: the final state depends on the actions
    env, prm, st, vel = _moving_box(3, seed=40)
    a, _ = O.rollout(env, prm, st, 3, vel=vel)
    b, _ = O.rollout(env, prm, st, 3, vel=vel + 0.5)
    assert (a[1] - b[1]).abs().max().item() > 1e-4


def test_action_gradient_matches_forward_mode():
    env, prm, st, vel = _moving_box(3, seed=41)
    S = 3
    rng = np.random.default_rng(42)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp, gvel, gc0 = O.rollout_vjp(env, prm, st, S, cot, vel=vel)
    assert gvel.abs().max().item() > 0
    zero = [torch.zeros_like(s) for s in st]
    for _ in range(3):
        tv = torch.from_numpy(rng.standard_normal((S, 3)))
        out = O.rollout_jvp(env, prm, st, S, zero, torch.zeros(7, dtype=DT), vel=vel, vel_tangent=tv)
        lhs = sum((a * b).sum() for a, b in zip(out, cot)).item()
        rhs = (gvel * tv).sum().item()
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs)), (lhs, rhs)


@pytest.mark.parametrize("edge", [False, True])
def test_action_and_start_gradients_match_central_differences(edge):
    import dataclasses
    env, prm, st, vel = _moving_box(3, seed=43, edge=edge)
    S = 3
    rng = np.random.default_rng(44)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp, gvel, gc0 = O.rollout_vjp(env, prm, st, S, cot, vel=vel)

    def loss(e, vv):
        (x, v, C, F), _ = O.rollout(e, prm, st, S, vel=vv)
        return sum((a * b).sum() for a, b in zip((x, v, C, F), cot)).item()

    for _ in range(3):
        tv = torch.from_numpy(rng.standard_normal((S, 3)))
        h = 1e-6
        fd = (loss(env, vel + h * tv) - loss(env, vel - h * tv)) / (2 * h)
        an = (gvel * tv).sum().item()
        assert abs(fd - an) <= 1e-5 * max(abs(an), abs(fd)) + 1e-9, (fd, an)
    # the starting center
    for a in range(3):
        h = 1e-7
        cp = list(env.collider.center); cm = list(env.collider.center)
        cp[a] += h; cm[a] -= h
        ep = dataclasses.replace(env, collider=dataclasses.replace(env.collider, center=tuple(cp)))
        em = dataclasses.replace(env, collider=dataclasses.replace(env.collider, center=tuple(cm)))
        fd = (loss(ep, vel) - loss(em, vel)) / (2 * h)
        an = gc0[a].item()
        assert abs(fd - an) <= 1e-5 * max(abs(an), abs(fd)) + 1e-8, (a, fd, an)


# ---------------------------------------------------------------- observation / reward moments
def test_moments_match_their_definitions():
    rng = np.random.default_rng(50)
    x = rng.uniform(0.2, 0.8, size=(500, 3))
    v = rng.standard_normal((500, 3))
    w = np.ones(500)
    m = O.moments(x, v, w).numpy()
    com, var_z, vbar = (t.numpy() if hasattr(t, "numpy") else t for t in O.moment_stats(torch.from_numpy(m)))
    np.testing.assert_allclose(com, x.mean(0), rtol=1e-13)
    np.testing.assert_allclose(var_z, x[:, 2].var(), rtol=1e-11)
    np.testing.assert_allclose(vbar, v.mean(0), rtol=1e-13)
    np.testing.assert_allclose(m[7], (x[:, 0] * x[:, 1]).sum(), rtol=1e-13)
    np.testing.assert_allclose(m[17], (v[:, 0] * v[:, 2]).sum(), rtol=1e-13)
    # a 0/1 weight pattern is the subsample itself
    sub = np.zeros(500)
    sub[::7] = 1.0
    np.testing.assert_allclose(O.moments(x, v, sub).numpy(), O.moments(x[::7], v[::7], np.ones(len(x[::7]))).numpy(),
                               rtol=1e-13)


# ---------------------------------------------------------------- the flip reward (HandFlip, Appendix E)
def test_pair_distance_hand_values_and_invariants():
    # two pairs at hand-computed distances 5 (a 3-4-5 triangle) and 2
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [1.0, 1.0, 1.0], [1.0, 1.0, 3.0]])
    pairs = np.array([[0, 1], [2, 3]])
    assert float(O.pair_distance(x, pairs)) == 3.5
    assert float(O.pair_distance(x, pairs[:, ::-1])) == 3.5          # symmetric in the pair order
    rng = np.random.default_rng(3)
    y = rng.uniform(size=(40, 3))
    p = rng.integers(0, 40, size=(25, 2))
    r = float(O.pair_distance(y, p))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    moved = y @ Q.T + rng.uniform(size=3)
    assert abs(float(O.pair_distance(moved, p)) - r) < 1e-14 * 10      # rigid motions leave it unchanged
    assert abs(float(O.pair_distance(2.5 * y, p)) - 2.5 * r) < 1e-14 * 10   # degree one in the positions


def test_mirror_pairs_of_a_symmetric_set_and_a_folded_one():
    # a lattice symmetric about z = 0.5: each lower particle is paired with its exact mirror image, and
    # folding the upper half onto the lower one (z -> 1 - z) brings the flip distance to zero
    g = np.arange(4) * 0.1 + 0.05
    lat = np.array([[a, b, c] for a in g for b in g for c in (0.25, 0.35, 0.45, 0.55, 0.65, 0.75)])
    pairs = O.mirror_pairs(lat, axis=2, plane=0.5)
    assert len(pairs) == len(lat) // 2
    lo, up = lat[pairs[:, 0]], lat[pairs[:, 1]]
    np.testing.assert_allclose(lo[:, :2], up[:, :2], atol=0)
    np.testing.assert_allclose(lo[:, 2] + up[:, 2], 1.0, atol=1e-15)
    # before folding: the mean of |z_u - z_l| over the pairs (0.5, 0.3, 0.1 for the three layers)
    assert abs(float(O.pair_distance(lat, pairs)) - 0.3) < 1e-15
    folded = lat.copy()
    upper = folded[:, 2] >= 0.5
    folded[upper, 2] = 1.0 - folded[upper, 2]
    assert float(O.pair_distance(folded, pairs)) < 1e-15


def test_normalized_improvement_clamps():
    r0 = torch.tensor(2.0, dtype=torch.float64)
    for r, want in ((2.0, 0.0), (1.0, 0.5), (0.0, 1.0), (4.0, -1.0), (9.0, -1.0)):
        assert float(O.normalized_improvement(torch.tensor(r, dtype=torch.float64), r0)) == want


def test_pair_distance_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    x = torch.from_numpy(rng.uniform(size=(30, 3))).requires_grad_(True)
    p = rng.integers(0, 30, size=(20, 2))
    p = p[p[:, 0] != p[:, 1]]
    O.pair_distance(x, p).backward()
    g = x.grad.numpy()
    # closed form: d/dx_a = (x_a - x_b) / ||x_a - x_b|| / P and the opposite for x_b
    want = np.zeros((30, 3))
    xv = x.detach().numpy()
    for a, b in p:
        u = (xv[a] - xv[b]) / np.linalg.norm(xv[a] - xv[b]) / len(p)
        want[a] += u
        want[b] -= u
    np.testing.assert_allclose(g, want, rtol=1e-12, atol=1e-15)
    h = 1e-6
    for i, c in ((3, 0), (7, 2), (11, 1)):
        xp, xm = xv.copy(), xv.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (float(O.pair_distance(xp, p)) - float(O.pair_distance(xm, p))) / (2 * h)
        assert abs(fd - g[i, c]) < 1e-8


# ---------------------------------------------------------------- a rotating box driven by angular-speed actions
def test_rotation_matrix_hand_values():
    R = O.rotation((0.0, 0.0, 1.0), math.pi / 2)
    np.testing.assert_allclose(R.numpy() @ np.array([1.0, 0.0, 0.0]), [0.0, 1.0, 0.0], atol=1e-15)
    a = np.array([1.0, 2.0, 2.0]) / 3.0
    R = O.rotation(tuple(a), 0.7).numpy()
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert abs(np.linalg.det(R) - 1.0) < 1e-15
    np.testing.assert_allclose(R @ a, a, atol=1e-15)          # the axis is fixed
    np.testing.assert_allclose(R.trace(), 1.0 + 2.0 * math.cos(0.7), atol=1e-15)   # rotation angle


def test_quarter_turned_box_is_the_axis_swapped_box():
    # a box turned by pi/2 about z is the axis-aligned box with its x and y half extents swapped:
    # same contact result at every node (nodes with ties between faces excluded: their normal picks
    # a face by index, which the turn relabels)
    n = 16
    turned = O.Box(center=(0.5, 0.5, 0.5), half=(0.1, 0.2, 0.15), velocity=(0.0, 0.0, 0.0), alpha=2.0 * n,
                   mu_b=0.5, angle=math.pi / 2)
    plain = O.Box(center=(0.5, 0.5, 0.5), half=(0.2, 0.1, 0.15), velocity=(0.0, 0.0, 0.0), alpha=2.0 * n, mu_b=0.5)
    rng = np.random.default_rng(5)
    v = torch.from_numpy(rng.standard_normal((n ** 3, 3)))
    act = torch.ones(n ** 3, dtype=torch.bool)
    rel = O.node_positions(n) - 0.5
    q = rel.abs() - torch.tensor([0.2, 0.1, 0.15], dtype=DT)
    top2 = q.topk(2, dim=1).values
    # also excluded: nodes on a symmetry plane (a zero component of x - c), where the side of the
    # normal is a convention that rounding of the turned frame (cos(pi/2) ~ 6e-17) can flip
    clear = ((top2[:, 0] - top2[:, 1]).abs() > 1e-9) & (rel.abs().min(dim=1).values > 1e-9)
    outs = []
    for box in (turned, plain):
        env = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=box)
        c, vb, th, om = O.collider_motion(env, 0.0)
        outs.append(O.collide(env, v, c, vb, act, th, om))
    np.testing.assert_allclose(outs[0][clear].numpy(), outs[1][clear].numpy(), atol=1e-12)
    assert int(clear.sum()) > 0.75 * n ** 3


def test_spinning_box_drags_nodes_inside_with_its_surface_velocity():
    # a node inside the box (s = 1) that sticks takes the box's velocity at that point, v_b + omega a x (x - c)
    n = 16
    box = O.Box(center=(0.5, 0.5, 0.5), half=(0.2, 0.2, 0.2), velocity=(0.1, 0.0, 0.0), alpha=2.0 * n, mu_b=10.0,
                axis=(0.0, 0.0, 1.0), angle=0.3, omega=4.0)
    env = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=box)
    pos = O.node_positions(n)
    i = int(((pos - torch.tensor([0.5625, 0.4375, 0.5], dtype=DT)).abs().sum(1)).argmin())
    v = torch.zeros(n ** 3, 3, dtype=DT)
    c, vb, th, om = O.collider_motion(env, 0.0)
    r = pos[i] - c
    vs = np.array([0.1, 0.0, 0.0]) + 4.0 * np.cross([0.0, 0.0, 1.0], r.numpy())
    d, nh = O.box_sdf(((pos - c) @ O.rotation(box.axis, th))[i:i + 1], torch.zeros(3, dtype=DT),
                      torch.tensor(box.half, dtype=DT))
    nw = (nh @ O.rotation(box.axis, th).T)[0].numpy()
    v[i] = torch.from_numpy(vs - 0.5 * nw)     # moving into the box along its normal: sticks (mu_b large)
    out = O.collide(env, v, c, vb, torch.ones(n ** 3, dtype=torch.bool), th, om)
    assert float(d[0]) < 0
    np.testing.assert_allclose(out[i].numpy(), vs, atol=1e-14)


def _spinning_box(S, seed):
    import dataclasses
    env, prm, st = tiny(O.FLUID_TAIT, collider=True)
    env = dataclasses.replace(env, collider=dataclasses.replace(env.collider, center=(0.6, 0.45, 0.45),
                                                                half=(0.05, 0.12, 0.2), axis=(0.0, 0.6, 0.8),
                                                                angle=0.4, omega=6.0, mu_b=0.3))
    rng = np.random.default_rng(seed)
    vel = torch.tensor(env.collider.velocity, dtype=DT) + 0.2 * torch.from_numpy(rng.standard_normal((S, 3)))
    om = 6.0 + 3.0 * torch.from_numpy(rng.standard_normal(S))
    return env, prm, st, vel, om


def test_constant_angular_actions_reproduce_the_spinning_box():
    env, prm, st, vel, _ = _spinning_box(4, seed=50)
    vel = torch.tensor(env.collider.velocity, dtype=DT).expand(4, 3).clone()
    a, _ = O.rollout(env, prm, st, 4)
    b, _ = O.rollout(env, prm, st, 4, vel=vel, omega=torch.full((4,), env.collider.omega, dtype=DT))
    for u, w in zip(a, b):
        np.testing.assert_allclose(u.numpy(), w.numpy(), rtol=0, atol=1e-12)
    c, ang = O.collider_path(env, vel, torch.full((4,), 6.0, dtype=DT))
    np.testing.assert_allclose(ang.numpy(), 0.4 + 6.0 * env.dt * np.arange(4), rtol=0, atol=1e-15)


def test_spin_actually_matters():
    env, prm, st, vel, om = _spinning_box(3, seed=51)
    a, _ = O.rollout(env, prm, st, 3, vel=vel, omega=om)
    b, _ = O.rollout(env, prm, st, 3, vel=vel, omega=om + 5.0)
    assert (a[1] - b[1]).abs().max().item() > 1e-4


def test_angular_action_gradients_match_forward_mode_and_central_differences():
    import dataclasses
    S = 3
    env, prm, st, vel, om = _spinning_box(S, seed=52)
    rng = np.random.default_rng(53)
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp, gvel, gc0, gom, gang0 = O.rollout_vjp(env, prm, st, S, cot, vel=vel, omega=om)
    assert gom.abs().max().item() > 0 and abs(gang0.item()) > 0
    zero = [torch.zeros_like(s) for s in st]
    for _ in range(3):
        tv = torch.from_numpy(rng.standard_normal((S, 3)))
        to = torch.from_numpy(rng.standard_normal(S))
        out = O.rollout_jvp(env, prm, st, S, zero, torch.zeros(7, dtype=DT), vel=vel, vel_tangent=tv, omega=om,
                            omega_tangent=to)
        lhs = sum((a * b).sum() for a, b in zip(out, cot)).item()
        rhs = (gvel * tv).sum().item() + (gom * to).sum().item()
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs)), (lhs, rhs)

    def loss(o=om, ang=None):
        e = env if ang is None else dataclasses.replace(env, collider=dataclasses.replace(env.collider, angle=ang))
        (x, v, C, F), _ = O.rollout(e, prm, st, S, vel=vel, omega=o)
        return sum((a * b).sum() for a, b in zip((x, v, C, F), cot)).item()

    h = 1e-6
    for k in range(S):
        op, omm = om.clone(), om.clone()
        op[k] += h
        omm[k] -= h
        fd = (loss(op) - loss(omm)) / (2 * h)
        assert abs(fd - gom[k].item()) <= 1e-5 * max(1.0, abs(fd)), (k, fd, gom[k].item())
    fd = (loss(ang=env.collider.angle + h) - loss(ang=env.collider.angle - h)) / (2 * h)
    assert abs(fd - gang0.item()) <= 1e-5 * max(1.0, abs(fd)), (fd, gang0.item())


def test_sphere_sdf_hand_values():
    # ball of radius 0.2 about c: points at 3-4-5 and 2-3-6-7 offsets, inside, and at the center
    c = torch.tensor([0.5, 0.5, 0.5], dtype=DT)
    cases = [
        ((0.15, 0.2, 0.0), 0.05, (0.6, 0.8, 0.0)),
        ((-0.06, 0.09, -0.18), 0.01, (-2 / 7, 3 / 7, -6 / 7)),
        ((0.0, 0.0, -0.05), -0.15, (0.0, 0.0, -1.0)),
        ((0.0, 0.0, 0.0), -0.2, (0.0, 0.0, 1.0)),          # the center: the normal is taken as +z
    ]
    p = c + torch.tensor([o for o, _, _ in cases], dtype=DT)
    d, nrm = O.sphere_sdf(p, c, 0.2)
    np.testing.assert_allclose(d.numpy(), [dd for _, dd, _ in cases], atol=1e-14)
    np.testing.assert_allclose(nrm.numpy(), [nn for _, _, nn in cases], atol=1e-14)


def test_sphere_contact_hand_values():
    # one node inside a static ball (s = 1) on its +x +y diagonal (normal (0.6, 0.8, 0)), moving in;
    # and the same ball spinning about z: its surface at the node moves at omega z x (x - c)
    n = 32
    r = 0.2
    ball = O.Box(center=(0.5, 0.5, 0.5), half=(r, r, r), velocity=(0.0, 0.0, 0.0), alpha=32.0, mu_b=0.5,
                 shape="sphere")
    env = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=ball)
    pos = O.node_positions(n)
    target = torch.tensor([0.5 + 0.09375, 0.5 + 0.125, 0.5], dtype=DT)   # |w| = 0.15625: inside, normal (0.6, 0.8, 0)
    i = int((pos - target).abs().sum(1).argmin())
    assert torch.allclose(pos[i], target, atol=1e-12)
    nrm = np.array([0.6, 0.8, 0.0])
    tang = np.array([-0.8, 0.6, 0.0])
    v = torch.zeros(n ** 3, 3, dtype=DT)
    act = torch.ones(n ** 3, dtype=torch.bool)
    cases = [(-1.0 * nrm + 0.2 * tang, np.zeros(3)),              # |u_t| = 0.2 <= 0.5: sticks
             (-1.0 * nrm + 2.0 * tang, 1.5 * tang),               # slides: u_t (1 - 0.5 * 1 / 2)
             (1.0 * nrm + 2.0 * tang, 1.0 * nrm + 2.0 * tang)]    # separating: unchanged
    for vin, vout in cases:
        v[i] = torch.tensor(vin, dtype=DT)
        out = O.collide(env, v, *O.collider_motion(env, 0.0)[:2], act)
        np.testing.assert_allclose(out[i].numpy(), vout, atol=1e-14)
    # spinning at omega about z: the surface velocity at the node is omega (-0.125, 0.09375, 0); a node at
    # rest relative to the world approaches nothing (u . n = 0) and keeps its velocity
    om = 4.0
    vs = om * np.array([-0.125, 0.09375, 0.0])
    v[i] = 0.0
    center, vb = O.collider_motion(env, 0.0)[:2]
    out = O.collide(env, v, center, vb, act, theta=0.7, omega=torch.tensor(om, dtype=DT))
    np.testing.assert_allclose(out[i].numpy(), vs + (-vs), atol=1e-14)   # u_n = 0: not approaching, unchanged
    v[i] = torch.tensor(-1.0 * nrm, dtype=DT)
    out = O.collide(env, v, center, vb, act, theta=0.7, omega=torch.tensor(om, dtype=DT))
    u = -1.0 * nrm - vs                       # relative velocity: u_n = -1, u_t = -vs (|u_t| = 0.625 > 0.5)
    ut = u - (u @ nrm) * nrm
    np.testing.assert_allclose(out[i].numpy(), vs + ut * (1.0 - 0.5 / np.linalg.norm(ut)), atol=1e-14)
    # the angle moves nothing: the same result at another angle
    out2 = O.collide(env, v, center, vb, act, theta=-2.1, omega=torch.tensor(om, dtype=DT))
    assert torch.equal(out, out2)


def test_capsule_contact_hand_values():
    # a capsule (box of half extents (0.15, 0, 0) rounded by 0.1) turned by 90 degrees about z, so its segment
    # runs along world y from c - 0.15 y to c + 0.15 y. Nodes (offsets from c, multiples of 1/32) beside the
    # segment and past its end: distance to the segment less 0.1, normal radial from the nearest segment point
    n = 32
    cap = O.Box(center=(0.5, 0.5, 0.5), half=(0.15, 0.0, 0.0), velocity=(0.0, 0.0, 0.0), alpha=32.0, mu_b=0.0,
                axis=(0.0, 0.0, 1.0), angle=math.pi / 2, rounding=0.1)
    env = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=cap)
    pos = O.node_positions(n)
    act = torch.ones(n ** 3, dtype=torch.bool)
    q_end = np.array([0.0625, 0.1875 - 0.15, 0.0])          # from the +y end point to the node
    cases = [
        ((0.0625, 0.09375, 0.0), 0.0625 - 0.1, (1.0, 0.0, 0.0)),             # beside the segment, inside
        ((0.0, -0.03125, -0.09375), 0.09375 - 0.1, (0.0, 0.0, -1.0)),        # beside the segment, inside
        ((0.125, 0.0, 0.0), 0.125 - 0.1, (1.0, 0.0, 0.0)),                   # beside the segment, outside
        ((0.0625, 0.1875, 0.0), float(np.linalg.norm(q_end)) - 0.1,           # past the +y end, inside
         tuple(q_end / np.linalg.norm(q_end))),
        ((0.0, -0.25, 0.0), 0.1 - 0.1, (0.0, -1.0, 0.0)),                    # on the -y cap's surface
    ]
    center, vb, th, om = O.collider_motion(env, 0.0)
    for off, dist, nrm in cases:
        i = int((pos - (center + torch.tensor(off, dtype=DT))).abs().sum(1).argmin())
        assert torch.allclose(pos[i], center + torch.tensor(off, dtype=DT), atol=1e-12)
        # moving into the capsule with no friction: the projected velocity keeps only the tangential part,
        # blended by s = min(exp(-alpha d), 1)
        nv = np.array(nrm)
        tang = np.cross(nv, [0.0, 0.0, 1.0]) if abs(nv[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        tang = tang / np.linalg.norm(tang)
        v = torch.zeros(n ** 3, 3, dtype=DT)
        v[i] = torch.tensor(-nv + 0.3 * tang, dtype=DT)
        out = O.collide(env, v, center, vb, act, th, om)[i].numpy()
        s = min(math.exp(-32.0 * dist), 1.0)
        np.testing.assert_allclose(out, s * 0.3 * tang + (1 - s) * (-nv + 0.3 * tang), atol=1e-13)


# ---------------------------------------------------------------- several colliders per env
def test_two_coincident_sticky_boxes_compose_their_blends():
    """Two identical static boxes with friction high enough to stick: a node
    approaching them ends at s vb + (1 - s) v after the first and at
    (1 - (1 - s)^2) vb + (1 - s)^2 v after both (vb = 0 here); a separating
    node keeps its velocity through both."""
    import dataclasses
    n = 16
    box = O.Box(center=(0.5, 0.5, 0.5), half=(0.2, 0.2, 0.2), velocity=(0.0, 0.0, 0.0), alpha=32.0, mu_b=50.0)
    one = O.Env(n=n, dt=1e-4, material=0, gravity=(0, 0, 0), collider=box)
    two = dataclasses.replace(one, more=(box,))
    pos = O.node_positions(n)
    i_out = int(((pos - torch.tensor([0.75, 0.5, 0.5], dtype=DT)).abs().sum(1)).argmin())   # d = 0.05, normal +x
    s = math.exp(-32.0 * 0.05)
    gm = torch.ones(n ** 3, dtype=DT)
    for vin, expect in [((-1.0, 0.2, 0.0), (1 - s) ** 2), ((1.0, 0.2, 0.0), 1.0)]:
        gP = torch.zeros(n ** 3, 3, dtype=DT)
        gP[i_out] = torch.tensor(vin, dtype=DT)
        v1 = O.grid_update(one, gm, gP, 0.0)
        v2 = O.grid_update(two, gm, gP, 0.0)
        if expect == 1.0:
            np.testing.assert_allclose(v2[i_out].numpy(), vin, atol=1e-14)
        else:
            np.testing.assert_allclose(v1[i_out].numpy(), (1 - s) * np.array(vin), atol=1e-14)
            np.testing.assert_allclose(v2[i_out].numpy(), expect * np.array(vin), atol=1e-14)


def test_far_apart_colliders_act_locally_and_in_order():
    """A box and a ball far apart (sharp blends): near each one the grid
    update with both equals the update with that one alone (the other's blend
    weight is below 1e-12 there); swapping their order changes nothing
    anywhere to that accuracy; nodes far from both keep the free velocity."""
    import dataclasses
    n = 24
    box = O.Box(center=(0.3, 0.5, 0.5), half=(0.08, 0.1, 0.06), velocity=(0.2, 0.0, -0.1), alpha=600.0, mu_b=0.4,
                axis=(0.0, 0.6, 0.8), angle=0.5, omega=3.0)
    ball = O.Box(center=(0.72, 0.5, 0.5), half=(0.07, 0.07, 0.07), velocity=(0.0, 0.3, 0.0), alpha=600.0, mu_b=0.2,
                 shape="sphere", omega=-2.0)
    rng = np.random.default_rng(3)
    gm = torch.from_numpy(rng.uniform(0.5, 2.0, n ** 3))
    gP = torch.from_numpy(rng.standard_normal((n ** 3, 3)))
    env_b = O.Env(n=n, dt=1e-4, material=0, collider=box)
    env_s = O.Env(n=n, dt=1e-4, material=0, collider=ball)
    both = O.Env(n=n, dt=1e-4, material=0, collider=box, more=(ball,))
    swapped = O.Env(n=n, dt=1e-4, material=0, collider=ball, more=(box,))
    t = 3e-4
    vb, vs, v2, vw = (O.grid_update(e, gm, gP, t) for e in (env_b, env_s, both, swapped))
    free = O.grid_update(O.Env(n=n, dt=1e-4, material=0), gm, gP, t)
    p = O.node_positions(n)
    near_box = (p[:, 0] < 0.5)
    near_ball = (p[:, 0] > 0.55)
    assert (vb - free)[near_box].abs().max() > 1e-2 and (vs - free)[near_ball].abs().max() > 1e-2
    np.testing.assert_allclose(v2[near_box].numpy(), vb[near_box].numpy(), atol=1e-12)
    np.testing.assert_allclose(v2[near_ball].numpy(), vs[near_ball].numpy(), atol=1e-12)
    np.testing.assert_allclose(v2.numpy(), vw.numpy(), atol=1e-12)
    assert dataclasses.replace(both).colliders == [box, ball]


def test_second_collider_action_gradients_match_central_differences():
    """Actions driving the second of two colliders (a static sticky box
    first, a ball pushed by the actions second): the reverse-mode cotangents
    of its velocities, angular speeds, start center and angle against central
    differences of the forward."""
    import dataclasses
    env, prm, st = tiny(O.FLUID_TAIT, collider=True)
    ball = O.Box(center=(0.45, 0.5, 0.42), half=(0.08, 0.08, 0.08), velocity=(0.0, 0.0, 0.0), alpha=40.0,
                 mu_b=0.3, shape="sphere")
    env = dataclasses.replace(env, more=(ball,))
    S = 3
    rng = np.random.default_rng(44)
    vel = 0.3 * torch.from_numpy(rng.standard_normal((S, 3)))
    om = torch.from_numpy(rng.standard_normal(S))
    cot = [torch.from_numpy(rng.standard_normal(s.shape)) for s in st]
    g, gp, gvel, gc0, gom, gang = O.rollout_vjp(env, prm, st, S, cot, vel=vel, omega=om, col=1)
    assert gvel.abs().max().item() > 0

    def loss(e, v_, o_):
        out, _ = O.rollout(e, prm, st, S, vel=v_, omega=o_, col=1)
        return sum((a * b).sum() for a, b in zip(out, cot)).item()

    h = 1e-6
    for _ in range(2):
        d = torch.from_numpy(rng.standard_normal((S, 3)))
        fd = (loss(env, vel + h * d, om) - loss(env, vel - h * d, om)) / (2 * h)
        assert (gvel * d).sum().item() == pytest.approx(fd, rel=1e-6, abs=1e-9)
    d = torch.from_numpy(rng.standard_normal(S))
    fd = (loss(env, vel, om + h * d) - loss(env, vel, om - h * d)) / (2 * h)
    assert (gom * d).sum().item() == pytest.approx(fd, rel=1e-6, abs=1e-9)
    dc = rng.standard_normal(3)
    shift = lambda sgn: dataclasses.replace(env, more=(dataclasses.replace(
        ball, center=tuple(np.array(ball.center) + sgn * h * dc)),))
    fd = (loss(shift(1), vel, om) - loss(shift(-1), vel, om)) / (2 * h)
    assert float(gc0 @ torch.from_numpy(dc)) == pytest.approx(fd, rel=1e-6, abs=1e-9)
