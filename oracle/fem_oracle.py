"""FP64 CPU oracle of the batched tetrahedral FEM substep with activations.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference that the
HIP FEM path is checked against. Only the test suite, the smoke check and the
bench's CPU-baseline leg may import it; the library never calls it. It shares
no code with the MPM oracle or with the library.

It follows the paper's Appendix D.2 ("Finite element method"): linear
tetrahedra, the stable neo-Hookean energy
    Psi(F) = mu/2 (I_C - 3) + lam/2 (J - alpha)^2 - mu/2 log(I_C + 1),
    I_C = tr(F^T F), J = det F,
integrated over each element, elastic forces from the energy gradient, and a
semi-implicit Euler step; the per-element actuation and the damping and
ground-contact terms the appendix names but does not write out follow the
readings below (each listed in the design notes):

* alpha = 1 + 3 mu / (4 lam), the value that makes the rest shape stress free;
* activation a_e of element e shifts the volume target: (J - alpha - a_e)^2,
  so a > 0 makes the element want to grow ("volumetric activations");
* damping is viscous in the deformation rate, first Piola stress k_damp dF/dt
  with dF/dt = D_v D_m^-1 (D_v the element's velocity differences);
* ground: a half-space z >= z_g with penalty contact on the nodes below it,
  normal force k_e (z_g - z) - k_d v_z and viscous friction -k_f (v_x, v_y);
* lumped masses: each element gives a quarter of rho W_e to each of its nodes;
* gravity (0, 0, -9.8); v' = v + dt (f / m + g), x' = x + dt v'.

Element e with nodes (i0, i1, i2, i3): D_m = [X1 - X0, X2 - X0, X3 - X0] at
rest, B_m = D_m^-1, W_e = |det D_m| / 6; F = D_s B_m with D_s the same
differences of the current positions; the forces on nodes i1..i3 are the
columns of H = -W_e P B_m^T and node i0 takes minus their sum, which is minus
the gradient of W_e Psi(F) in the node positions.

Gradients are the discrete adjoint of the step (Appendix D's simulation
gradient): reverse mode from torch autograd through the forward as written,
forward mode from torch's dual numbers through the same code.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

DT = torch.float64
GRAVITY = (0.0, 0.0, -9.8)
# per-env parameters, in this order
FEM_PARAMS = ("mu", "lam", "rho", "damp", "ke", "kd", "kf", "ground")


@dataclass
class Mesh:
    """Shared topology of a batch: tets [T, 4] node indices."""
    tets: np.ndarray


def alpha(mu, lam):
    """Volume target of the stable neo-Hookean energy that makes F = I stress free."""
    return 1.0 + 0.75 * mu / lam


def cofactor(F):
    """cof(F) = dJ/dF from the columns f0, f1, f2 of F: its columns are
    f1 x f2, f2 x f0 and f0 x f1 (each the gradient of det F = f0 . (f1 x f2)
    in one column)."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    return torch.stack([torch.linalg.cross(f1, f2), torch.linalg.cross(f2, f0), torch.linalg.cross(f0, f1)], dim=-1)


def energy_density(F, mu, lam, a):
    """Psi(F) with the activation shift (Appendix D.2's energy, reading above)."""
    Ic = (F * F).sum((-2, -1))
    J = torch.linalg.det(F)
    return 0.5 * mu * (Ic - 3.0) + 0.5 * lam * (J - alpha(mu, lam) - a) ** 2 - 0.5 * mu * torch.log(Ic + 1.0)


def piola(F, Fdot, mu, lam, damp, a):
    """First Piola stress dPsi/dF plus the viscous damping term:
    P = mu (1 - 1/(I_C + 1)) F + lam (J - alpha - a) cof(F) + damp dF/dt."""
    Ic = (F * F).sum((-2, -1))
    J = torch.linalg.det(F)
    s = mu * (1.0 - 1.0 / (Ic + 1.0))
    return s[..., None, None] * F + (lam * (J - alpha(mu, lam) - a))[..., None, None] * cofactor(F) + damp * Fdot


def rest_data(X, tets):
    """(B_m [T, 3, 3], W [T], lumped mass per unit density [n]) of rest positions X [n, 3]."""
    X = torch.as_tensor(X, dtype=DT)
    t = torch.as_tensor(np.asarray(tets), dtype=torch.long)
    Dm = torch.stack([X[t[:, 1]] - X[t[:, 0]], X[t[:, 2]] - X[t[:, 0]], X[t[:, 3]] - X[t[:, 0]]], dim=-1)
    Bm = torch.linalg.inv(Dm)
    W = torch.abs(torch.linalg.det(Dm)) / 6.0
    w = torch.zeros(X.shape[0], dtype=DT)
    for c in range(4):
        w = w.index_add(0, t[:, c], W / 4.0)
    return Bm, W, w


def elastic_forces(x, v, tets, Bm, W, prm, a):
    """Element forces (elasticity, activation, damping) summed on the nodes."""
    t = torch.as_tensor(np.asarray(tets), dtype=torch.long)
    mu, lam, damp = prm[0], prm[1], prm[3]
    Ds = torch.stack([x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]], x[t[:, 3]] - x[t[:, 0]]], dim=-1)
    Dv = torch.stack([v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]], v[t[:, 3]] - v[t[:, 0]]], dim=-1)
    F = Ds @ Bm
    Fdot = Dv @ Bm
    P = piola(F, Fdot, mu, lam, damp, a)
    H = -W[:, None, None] * (P @ Bm.transpose(-1, -2))
    f = torch.zeros_like(x)
    f = f.index_add(0, t[:, 1], H[:, :, 0])
    f = f.index_add(0, t[:, 2], H[:, :, 1])
    f = f.index_add(0, t[:, 3], H[:, :, 2])
    f = f.index_add(0, t[:, 0], -(H[:, :, 0] + H[:, :, 1] + H[:, :, 2]))
    return f


def ground_forces(x, v, prm):
    """Penalty contact with the half-space z >= ground on the nodes below it."""
    ke, kd, kf, zg = prm[4], prm[5], prm[6], prm[7]
    pen = x[:, 2] < zg
    fz = ke * (zg - x[:, 2]) - kd * v[:, 2]
    f = torch.stack([-kf * v[:, 0], -kf * v[:, 1], fz], dim=1)
    return torch.where(pen[:, None], f, torch.zeros_like(f))


def substep(mesh: Mesh, Bm, W, wmass, prm, x, v, a, dt: float):
    """One semi-implicit Euler step: v' = v + dt (f/m + g), x' = x + dt v'."""
    f = elastic_forces(x, v, mesh.tets, Bm, W, prm, a) + ground_forces(x, v, prm)
    m = prm[2] * wmass
    g = torch.tensor(GRAVITY, dtype=DT)
    v1 = v + dt * (f / m[:, None] + g)
    x1 = x + dt * v1
    return x1, v1


def rollout(mesh: Mesh, X, prm, x0, v0, act, S: int, dt: float, keep_all: bool = False):
    """S substeps from (x0, v0) with activations act [>= S, T]; returns the final
    state (and every state if keep_all)."""
    prm = torch.as_tensor(prm, dtype=DT)
    Bm, W, wmass = rest_data(X, mesh.tets)
    x, v = torch.as_tensor(x0, dtype=DT), torch.as_tensor(v0, dtype=DT)
    act = torch.as_tensor(act, dtype=DT)
    states = [(x, v)]
    for k in range(S):
        x, v = substep(mesh, Bm, W, wmass, prm, x, v, act[k], dt)
        if keep_all:
            states.append((x, v))
    return (x, v, states) if keep_all else (x, v)


def rollout_vjp(mesh: Mesh, X, prm, x0, v0, act, S: int, dt: float, gx, gv):
    """Reverse mode through rollout: cotangents of (x0, v0, act[:S], prm[8]) for
    the output cotangents (gx, gv)."""
    x0 = torch.as_tensor(x0, dtype=DT).clone().requires_grad_(True)
    v0 = torch.as_tensor(v0, dtype=DT).clone().requires_grad_(True)
    act = torch.as_tensor(act, dtype=DT)[:S].clone().requires_grad_(True)
    prm = torch.as_tensor(prm, dtype=DT).clone().requires_grad_(True)
    x, v = rollout(mesh, X, prm, x0, v0, act, S, dt)
    L = (x * torch.as_tensor(gx, dtype=DT)).sum() + (v * torch.as_tensor(gv, dtype=DT)).sum()
    if not L.requires_grad:   # S = 0 and no dependence on act or prm
        return (torch.as_tensor(gx, dtype=DT), torch.as_tensor(gv, dtype=DT), torch.zeros_like(act),
                torch.zeros_like(prm))
    g = torch.autograd.grad(L, (x0, v0, act, prm), allow_unused=True)
    return tuple(torch.zeros_like(t) if gi is None else gi for gi, t in zip(g, (x0, v0, act, prm)))


def rollout_jvp(mesh: Mesh, X, prm, x0, v0, act, S: int, dt: float, tangents):
    """Forward mode through rollout: the tangent of (x_S, v_S) for tangents of
    (x0, v0, act, prm) given as a 4-tuple."""
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        duals = [fwAD.make_dual(torch.as_tensor(p, dtype=DT), torch.as_tensor(t, dtype=DT))
                 for p, t in zip((x0, v0, act, prm), tangents)]
        x, v = rollout(mesh, X, duals[3], duals[0], duals[1], duals[2], S, dt)
        return fwAD.unpack_dual(x).tangent, fwAD.unpack_dual(v).tangent
