"""FP64 CPU oracle of the differentiable MLS-MPM substep.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference that the
HIP path is checked against. Only the test suite, the smoke check and the
bench's CPU-baseline leg may import it; the library never calls it.

It follows the paper's Appendix D.3 ("Material point method"): MLS-MPM with
APIC transfer (Hu et al. 2018, cited there), the von Mises elastoplastic law
with Hencky strain and its return mapping, the weakly compressible fluid with
the J^(1/3) projection, the softened one-way rigid-to-MPM contact blend; and
the stable neo-Hookean energy of Appendix D.2 used as a per-particle material.
Gradients are the discrete adjoint of Appendix D ("simulation gradient"
chain): reverse mode comes from torch autograd through the forward as written,
forward mode from torch's dual numbers through the same code. Nothing here is
blocked, fused or reordered beyond the equations.

Readings where the paper is silent or garbled (each listed in the design notes):
* quadratic B-spline kernel, base = floor(x n - 1/2), D^-1 = 4 n^2 (MLS-MPM);
* nodes at i/n, i = 0..n-1, on the unit cube; sticky walls 3 nodes thick;
* gravity (0, 0, -9.8) applied on the grid (z up, Appendix E notation);
* stress from the stored (already projected) F; F updated in G2P with the new C;
* elastoplastic stress read as Kirchhoff tau = U (2 mu eps + lam tr(eps) I) U^T
  with eps = log(Sigma); the yield offset follows the printed 2 sigma_y / (2 mu)
  (``YIELD_SCALE = 2``);
* fluid: Tait pressure p = K (J^-gamma - 1), tau = -J p I ("fluid_tait"), or the
  printed lam J (J - 1) I ("fluid_paper"); both project F to J^(1/3) I;
* neo-Hookean alpha = 1 + 3 mu / (4 lam) so that tau(I) = 0;
* contact: box SDF, s = min(exp(-alpha d), 1), Coulomb projection of the
  velocity relative to the box, blended by s; applied where node mass > 0.

Branch conventions of the derivative (all hold the primal's branch): floor and
the base clamp have derivative 0; the m > 0 test, the wall mask, the von Mises
yield test and the contact/friction cases are fixed at the primal.

Matrix functions use textbook algorithms that are smooth in their argument, so
autograd and dual numbers differentiate them without eigen-decompositions:
polar factor by Newton's iteration X <- (X + X^-T)/2; matrix square root by the
Denman-Beavers iteration; matrix log by inverse scaling and squaring with the
series log(B) = 2 atanh((B - I)(B + I)^-1); matrix exp by scaling and squaring
of the Taylor series (Higham, "Functions of Matrices", 2008).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

DT = torch.float64

NEOHOOKEAN, COROTATED, VONMISES, FLUID_TAIT, FLUID_PAPER = range(5)
YIELD_SCALE = 2.0          # printed numerator of the yield offset: YIELD_SCALE * sigma_y / (2 mu)
SIGMA_MIN = 1e-4           # singular values are clamped below this before the log
PARAM_NAMES = ("E", "nu", "rho", "Vp", "sigma_y", "K", "gamma")

# the 27 stencil offsets, x-major (ox, oy, oz)
OFFSETS = torch.tensor([[a, b, c] for a in range(3) for b in range(3) for c in range(3)], dtype=DT)


@dataclass
class Box:
    center: Tuple[float, float, float]
    half: Tuple[float, float, float]       # half extents along the box's own axes
    velocity: Tuple[float, float, float]
    alpha: float
    mu_b: float
    axis: Tuple[float, float, float] = (0.0, 0.0, 1.0)   # unit rotation axis (world)
    angle: float = 0.0                     # rotation about the axis at t = 0 (rad)
    omega: float = 0.0                     # constant angular speed about the axis (rad/s)
    shape: str = "box"                     # "box", or "sphere": a ball of radius half[0] about the center
    rounding: float = 0.0                  # a box's distance less this radius: a rounded box (half (h, 0, 0):
                                           # a capsule along the box's x axis)


@dataclass
class Env:
    """Fixed (non-differentiated) settings of one environment."""
    n: int
    dt: float
    material: int
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.8)
    wall: int = 3
    collider: Optional[Box] = None
    more: Tuple[Box, ...] = ()   # further colliders, applied after the first one, in order

    @property
    def colliders(self) -> List[Box]:
        """Every collider of the env in the order the grid update applies them."""
        return ([self.collider] if self.collider is not None else []) + list(self.more)


def _box_from(c) -> Box:
    return Box(tuple(c.center), tuple(c.half), tuple(c.velocity), float(c.alpha), float(c.mu_b),
               tuple(getattr(c, "axis", (0.0, 0.0, 1.0))), float(getattr(c, "angle", 0.0)),
               float(getattr(c, "omega", 0.0)), str(getattr(c, "shape", "box")), float(getattr(c, "rounding", 0.0)))


def env_from_spec(spec) -> Tuple[Env, torch.Tensor, Tuple[torch.Tensor, ...]]:
    """Convert a scene EnvSpec into (Env, params[7], state) in float64."""
    box = None if spec.collider is None else _box_from(spec.collider)
    more = tuple(_box_from(c) for c in getattr(spec, "more_colliders", ()))
    env = Env(n=spec.n, dt=spec.dt, material=spec.material, gravity=tuple(spec.gravity),
              wall=spec.wall, collider=box, more=more)
    prm = torch.tensor([spec.E, spec.nu, spec.rho, spec.Vp, spec.sigma_y, spec.K, spec.gamma], dtype=DT)
    st = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).to(DT) for a in (spec.x, spec.v, spec.C, spec.F))
    return env, prm, st


# ----------------------------------------------------------------------------
# a1: parameter preparation (textbook Lame parameters from E, nu)
# ----------------------------------------------------------------------------
def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson's ratio."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


# ----------------------------------------------------------------------------
# 3x3 helpers
# ----------------------------------------------------------------------------
def eye_like(A):
    return torch.eye(3, dtype=A.dtype).expand(A.shape).clone() if A.dim() > 2 else torch.eye(3, dtype=A.dtype)


def tr(A):
    return A.diagonal(dim1=-2, dim2=-1).sum(-1)


def polar_rotation(F, tol=1e-15, max_iter=100):
    """Rotation factor R of F = R S by Newton's iteration X <- (X + X^-T)/2 (Higham 1986)."""
    X = F
    for _ in range(max_iter):
        Xn = 0.5 * (X + torch.linalg.inv(X).transpose(-1, -2))
        done = (Xn.detach() - X.detach()).abs().max().item() <= tol
        X = Xn
        if done:
            break
    # two more sweeps so the tangent has converged as well as the value
    for _ in range(2):
        X = 0.5 * (X + torch.linalg.inv(X).transpose(-1, -2))
    return X


def sqrtm_spd(B, tol=1e-15, max_iter=100):
    """Principal square root of SPD matrices by the Denman-Beavers iteration."""
    Y, Z = B, eye_like(B)
    for _ in range(max_iter):
        Yn = 0.5 * (Y + torch.linalg.inv(Z))
        Zn = 0.5 * (Z + torch.linalg.inv(Y))
        done = (Yn.detach() - Y.detach()).abs().max().item() <= tol * max(1.0, Y.detach().abs().max().item())
        Y, Z = Yn, Zn
        if done:
            break
    for _ in range(2):
        Y, Z = 0.5 * (Y + torch.linalg.inv(Z)), 0.5 * (Z + torch.linalg.inv(Y))
    return Y


def logm_spd(B, n_terms=14):
    """Matrix logarithm of SPD matrices: inverse scaling and squaring + atanh series.

    Square roots are taken until every eigenvalue lies within 1/4 of 1 (checked
    through the Frobenius norm of B - I), then log(B) = 2 sum_k Z^(2k+1)/(2k+1)
    with Z = (B - I)(B + I)^-1, and the result is scaled back by 2^s.
    """
    I = eye_like(B)
    s = 0
    X = B
    while (X.detach() - I).flatten(-2).norm(dim=-1).max().item() > 0.25 and s < 60:
        X = sqrtm_spd(X)
        s += 1
    Z = (X - I) @ torch.linalg.inv(X + I)
    Z2 = Z @ Z
    term = Z
    acc = Z.clone()
    for k in range(1, n_terms):
        term = term @ Z2
        acc = acc + term / (2 * k + 1)
    return (2.0 ** (s + 1)) * acc


def expm_sym(X, n_terms=22):
    """Matrix exponential by scaling and squaring of the Taylor series."""
    nrm = X.detach().flatten(-2).norm(dim=-1).max().item() if X.numel() else 0.0
    s = max(0, int(math.ceil(math.log2(nrm / 0.25)))) if nrm > 0.25 else 0
    Y = X / (2.0 ** s)
    I = eye_like(X)
    term = I
    acc = I.clone()
    for k in range(1, n_terms):
        term = term @ Y / k
        acc = acc + term
    for _ in range(s):
        acc = acc @ acc
    return acc


# ----------------------------------------------------------------------------
# a2: binning keys and the stable particle order (bit-exact interface)
# ----------------------------------------------------------------------------
def base_cells(x32: np.ndarray, n: int) -> np.ndarray:
    """Stencil base per axis, floor(x n - 1/2), evaluated exactly in float64 for float32 x."""
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    return np.floor(x * n - 0.5).astype(np.int64)


def base_cells_exact(x32: np.ndarray, n: int) -> np.ndarray:
    """Same as base_cells with exact rational arithmetic (for pinning on small inputs)."""
    out = np.empty(np.shape(x32), dtype=np.int64)
    flat_in = np.asarray(x32, dtype=np.float32).reshape(-1)
    flat_out = out.reshape(-1)
    for i, xv in enumerate(flat_in):
        q = Fraction(float(xv)) * n - Fraction(1, 2)
        flat_out[i] = math.floor(q)
    return out


def cell_keys(x32: np.ndarray, n: int) -> np.ndarray:
    """Sort key of each particle: 4^3-node tile (raster order) then cell inside the tile.

    base is clamped to [0, n-3] first; key = tile * 64 + cell, with
    tile = ((bx/4) T + by/4) T + bz/4, T = n/4, cell = ((bx%4) 4 + by%4) 4 + bz%4.
    """
    b = np.clip(base_cells(x32, n), 0, n - 3)
    T = n // 4
    t = ((b[:, 0] // 4) * T + (b[:, 1] // 4)) * T + (b[:, 2] // 4)
    c = ((b[:, 0] % 4) * 4 + (b[:, 1] % 4)) * 4 + (b[:, 2] % 4)
    return (t * 64 + c).astype(np.int64)


def sort_permutation(keys: np.ndarray) -> np.ndarray:
    """Stable argsort: the new position j holds the particle at old position perm[j]."""
    return np.argsort(keys, kind="stable").astype(np.int64)


# ----------------------------------------------------------------------------
# a3: Kirchhoff stress tau = P F^T per material
# ----------------------------------------------------------------------------
def stress(material: int, F, mu, lam, K, gamma):
    """Kirchhoff stress of each particle from its stored deformation gradient."""
    I = eye_like(F)
    J = torch.linalg.det(F)
    if material == NEOHOOKEAN:
        # stable neo-Hookean energy (Appendix D.2): P = mu (1 - 1/(I_C+1)) F + lam (J - alpha) J F^-T
        b = F @ F.transpose(-1, -2)
        Ic = tr(b)
        alpha = 1.0 + 3.0 * mu / (4.0 * lam)
        return (mu * (1.0 - 1.0 / (Ic + 1.0)))[..., None, None] * b + (lam * J * (J - alpha))[..., None, None] * I
    if material == COROTATED:
        R = polar_rotation(F)
        return 2.0 * mu * (F - R) @ F.transpose(-1, -2) + (lam * J * (J - 1.0))[..., None, None] * I
    if material == VONMISES:
        # Hencky: tau = U (2 mu log Sigma + lam tr(log Sigma) I) U^T = mu log(F F^T) + lam log(J) I
        b = F @ F.transpose(-1, -2)
        ev = torch.linalg.eigvalsh(b.detach())
        if ev.numel() and ev.min().item() < SIGMA_MIN ** 2:
            raise ValueError("singular value below SIGMA_MIN: clamp branch is not modelled by the oracle")
        return mu * logm_spd(b) + (lam * torch.log(J))[..., None, None] * I
    if material == FLUID_TAIT:
        p = K * (J ** (-gamma) - 1.0)
        return (-J * p)[..., None, None] * I
    if material == FLUID_PAPER:
        # P = lam J (J - 1) F^-T  =>  tau = lam J (J - 1) I
        return (lam * J * (J - 1.0))[..., None, None] * I
    raise ValueError(f"unknown material {material}")


# ----------------------------------------------------------------------------
# a6 (second half): plasticity projection of the trial deformation gradient
# ----------------------------------------------------------------------------
def project(material: int, Ftr, mu, sigma_y):
    """Return mapping P(F_tr) of Appendix D.3."""
    if material in (NEOHOOKEAN, COROTATED):
        return Ftr
    if material in (FLUID_TAIT, FLUID_PAPER):
        J = torch.linalg.det(Ftr)
        return (torch.sign(J) * J.abs() ** (1.0 / 3.0))[..., None, None] * eye_like(Ftr)
    if material == VONMISES:
        if Ftr.shape[0] == 0:
            return Ftr
        # eps = log Sigma as the matrix (1/2) log(F F^T); eps_hat its deviatoric part
        b = Ftr @ Ftr.transpose(-1, -2)
        Y = YIELD_SCALE * sigma_y / (2.0 * mu)
        with torch.no_grad():
            eps = 0.5 * logm_spd(b)
            eps_hat = eps - (tr(eps) / 3.0)[..., None, None] * eye_like(eps)
            plastic = (eps_hat.flatten(-2).norm(dim=-1) - Y) > 0
        idx = plastic.nonzero().flatten()
        if idx.numel() == 0:
            return Ftr
        Fp = Ftr[idx]
        eps = 0.5 * logm_spd(b[idx])
        eps_hat = eps - (tr(eps) / 3.0)[..., None, None] * eye_like(eps)
        nrm = eps_hat.flatten(-2).norm(dim=-1)
        dgam = nrm - Y
        # U exp(eps - dgam eps_hat/|eps_hat|) V^T = exp(-dgam/|eps_hat| eps_hat) F_tr
        Fnew = expm_sym(-(dgam / nrm)[..., None, None] * eps_hat) @ Fp
        return Ftr.index_put((idx,), Fnew)
    raise ValueError(f"unknown material {material}")


# ----------------------------------------------------------------------------
# transfer pieces
# ----------------------------------------------------------------------------
def stencil(x, n: int):
    """Base node, quadratic B-spline weights and node offsets d = (o - f) dx of each particle.

    Returns (base [N,3] int64, W [N,27], d [N,27,3], out_of_band [N] bool).
    """
    with torch.no_grad():
        base = torch.floor(x.detach() * n - 0.5)
        oob = ((base < 0) | (base > n - 3)).any(dim=1)
        base = base.clamp(0, n - 3)
    f = x * n - base
    w = torch.stack([0.5 * (1.5 - f) ** 2, 0.75 - (f - 1.0) ** 2, 0.5 * (f - 0.5) ** 2], dim=1)  # [N,3o,3ax]
    o = OFFSETS.long()
    W = w[:, o[:, 0], 0] * w[:, o[:, 1], 1] * w[:, o[:, 2], 2]
    d = (OFFSETS[None, :, :] - f[:, None, :]) / n
    return base.long(), W, d, oob


def node_index(base, n: int):
    node = base[:, None, :] + OFFSETS.long()[None, :, :]
    return (node[..., 0] * n + node[..., 1]) * n + node[..., 2]


def p2g(env: Env, prm, x, v, C, F):
    """a3+a4: scatter particle mass and APIC momentum with the MLS stress impulse.

    m_i = sum_p w m_p;  P_i = sum_p w (m_p v_p + A_p d),  A_p = -dt V_p 4 n^2 tau_p + m_p C_p.
    """
    E, nu, rho, Vp, sy, K, gam = prm.unbind()
    mu, lam = lame(E, nu)
    mp = rho * Vp
    n = env.n
    base, W, d, oob = stencil(x, n)
    tau = stress(env.material, F, mu, lam, K, gam)
    A = (-env.dt * 4.0 * n * n) * Vp * tau + mp * C
    lin = node_index(base, n).reshape(-1)
    gm = torch.zeros(n ** 3, dtype=DT).index_add(0, lin, (W * mp).reshape(-1))
    mom = W[..., None] * (mp * v[:, None, :] + torch.einsum("pij,pkj->pki", A, d))
    gP = torch.zeros(n ** 3, 3, dtype=DT).index_add(0, lin, mom.reshape(-1, 3))
    return gm, gP, oob


def node_positions(n: int):
    i = torch.arange(n, dtype=DT) / n
    return torch.stack(torch.meshgrid(i, i, i, indexing="ij"), dim=-1).reshape(-1, 3)


def wall_mask(n: int, wall: int):
    i = torch.arange(n)
    g = torch.stack(torch.meshgrid(i, i, i, indexing="ij"), dim=-1).reshape(-1, 3)
    return ((g < wall) | (g > n - 1 - wall)).any(dim=1)


def box_sdf(p, center, half):
    """Signed distance to an axis-aligned box and its outward unit normal (gradient)."""
    rel = p - center
    q = rel.abs() - half
    qpos = q.clamp(min=0.0)
    out_len = qpos.norm(dim=1)
    inside = q.max(dim=1).values
    d = out_len + inside.clamp(max=0.0)
    sgn = torch.where(rel >= 0, 1.0, -1.0).to(DT)
    outside = out_len > 0
    n_out = sgn * qpos / torch.where(outside, out_len, 1.0)[:, None]
    ax = q.argmax(dim=1)
    n_in = torch.nn.functional.one_hot(ax, 3).to(DT) * sgn
    nrm = torch.where(outside[:, None], n_out, n_in)
    return d, nrm


def sphere_sdf(p, center, radius):
    """Signed distance to a ball, |p - c| - r, and its outward unit normal
    (p - c) / |p - c| (the +z axis at the center itself, where it is undefined)."""
    rel = p - center
    L = rel.norm(dim=1)
    at_c = L == 0
    nrm = torch.where(at_c[:, None], torch.tensor([0.0, 0.0, 1.0], dtype=DT), rel / torch.where(at_c, 1.0, L)[:, None])
    return L - radius, nrm


def rotation(axis, theta):
    """Rotation by theta about the unit axis (Rodrigues): I + sin t K + (1 - cos t) K^2, K = [axis]x."""
    a = torch.as_tensor(axis, dtype=DT)
    K = torch.zeros(3, 3, dtype=DT)
    K[0, 1], K[0, 2], K[1, 0], K[1, 2], K[2, 0], K[2, 1] = -a[2], a[1], a[2], -a[0], -a[1], a[0]
    theta = torch.as_tensor(theta, dtype=DT)
    return torch.eye(3, dtype=DT) + torch.sin(theta) * K + (1.0 - torch.cos(theta)) * (K @ K)


def collide(env: Env, v, center, vb, active, theta=0.0, omega=0.0, box: Optional[Box] = None):
    """Softened one-way contact (Appendix D.3): blend pre/post projection by s = min(exp(-alpha d), 1).

    ``center``, ``vb``, ``theta`` and ``omega`` are the box's center, velocity,
    rotation angle about its axis and angular speed during this substep
    (tensors, so that derivatives reach a prescribed collider motion). The box
    is axis-aligned in its own frame: a node's distance and normal come from
    its position R^T (x - c) in that frame, rotated back to the world, and the
    box surface moves at vb + omega axis x (x - c). A sphere collider's
    distance and normal do not depend on its angle; its spin still moves its
    surface. A rounded box's distance is the box's less the rounding radius,
    its normal the box's. ``box`` defaults to the env's first collider."""
    box = env.collider if box is None else box
    n = env.n
    p = node_positions(n)
    if box.shape == "sphere":
        d, nh = sphere_sdf(p, center, float(box.half[0]))
    else:
        R = rotation(box.axis, theta)
        d, nh = box_sdf((p - center) @ R, torch.zeros(3, dtype=DT), torch.tensor(box.half, dtype=DT))
        d = d - box.rounding
        nh = nh @ R.T
    a = torch.tensor(box.axis, dtype=DT)
    vb = vb + omega * torch.linalg.cross(a.expand_as(p), p - center)
    s = torch.clamp(torch.exp(-box.alpha * d), max=1.0)
    u = v - vb
    un = (u * nh).sum(1)
    ut = u - un[:, None] * nh
    utn = ut.norm(dim=1)
    approaching = un < 0
    stick = approaching & (utn <= -box.mu_b * un)
    slide = approaching & ~stick
    idx = slide.nonzero().flatten()
    u_proj = torch.where(stick[:, None], torch.zeros_like(u), u)
    if idx.numel():
        ut_s, utn_s, un_s = ut[idx], utn[idx], un[idx]
        u_proj = u_proj.index_put((idx,), ut_s * (1.0 + box.mu_b * un_s / utn_s)[:, None])
    s_eff = torch.where(active, s, torch.zeros_like(s))[:, None]
    return s_eff * (vb + u_proj) + (1.0 - s_eff) * v


def collider_motion(env: Env, t: float, motion=None, box: Optional[Box] = None):
    """(center, velocity, angle, angular speed) of the box during the substep
    that starts at time t.

    Without a prescribed motion the box moves at its constant velocity and
    angular speed: center = c0 + t v_b, angle = angle0 + t omega. With one,
    ``motion`` is this substep's (center, v_b, angle, omega) from
    collider_path."""
    if motion is not None:
        return motion
    box = env.collider if box is None else box
    vb = torch.tensor(box.velocity, dtype=DT)
    om = torch.tensor(box.omega, dtype=DT)
    return torch.tensor(box.center, dtype=DT) + t * vb, vb, box.angle + t * om, om


def collider_path(env: Env, vel, omega=None, col: int = 0):
    """Centers (and angles) of collider `col` driven by per-substep velocities
    vel [S, 3] and angular speeds omega [S] (the actions): during substep k the
    center is c0 + dt sum_{j<k} vel_j and the angle angle0 + dt sum_{j<k} omega_j."""
    box = env.colliders[col]
    c0 = torch.tensor(box.center, dtype=DT)
    steps = torch.cat([torch.zeros(1, 3, dtype=vel.dtype), env.dt * vel[:-1]], 0)
    centers = c0 + torch.cumsum(steps, 0)
    if omega is None:
        return centers
    ast = torch.cat([torch.zeros(1, dtype=omega.dtype), env.dt * omega[:-1]], 0)
    return centers, box.angle + torch.cumsum(ast, 0)


def grid_update(env: Env, gm, gP, t: float, motion=None):
    """a5: v = P/m + dt g where m > 0 (else 0), contact blend with each
    collider in turn (each one's output feeds the next), then sticky walls.
    ``motion``: None, one collider's (center, v_b, angle, omega) for the first
    collider, or a list with such an entry (or None) per collider."""
    g = torch.tensor(env.gravity, dtype=DT)
    pos = gm > 0
    msafe = torch.where(pos, gm, torch.ones_like(gm))
    v = torch.where(pos[:, None], gP / msafe[:, None] + env.dt * g, torch.zeros_like(gP))
    motions = motion if isinstance(motion, list) else [motion]
    for ci, box in enumerate(env.colliders):
        mo = motions[ci] if ci < len(motions) else None
        center, vb, theta, om = collider_motion(env, t, mo, box)
        v = collide(env, v, center, vb, pos, theta, om, box)
    wm = wall_mask(env.n, env.wall)
    return torch.where(wm[:, None], torch.zeros_like(v), v)


def g2p(env: Env, prm, x, F, gv):
    """a6: gather velocity and APIC affine field, advect, update and project F."""
    E, nu, rho, Vp, sy, K, gam = prm.unbind()
    mu, lam = lame(E, nu)
    n = env.n
    base, W, d, _ = stencil(x, n)
    vi = gv[node_index(base, n)]                      # [N,27,3]
    vn = (W[..., None] * vi).sum(1)
    Cn = (4.0 * n * n) * torch.einsum("pk,pki,pkj->pij", W, vi, d)
    xn = x + env.dt * vn
    Ftr = (eye_like(F) + env.dt * Cn) @ F
    Fn = project(env.material, Ftr, mu, sy)
    return xn, vn, Cn, Fn


def substep(env: Env, prm, x, v, C, F, t: float, motion=None):
    """One MLS-MPM substep of one environment: P2G, grid update, G2P."""
    gm, gP, oob = p2g(env, prm, x, v, C, F)
    gv = grid_update(env, gm, gP, t, motion)
    xn, vn, Cn, Fn = g2p(env, prm, x, F, gv)
    return xn, vn, Cn, Fn, bool(oob.any().item())


def motion_path(env: Env, vel, omega=None, col: int = 0):
    """Per-substep (center, velocity, angle, angular speed) of collider `col`
    driven by actions: velocities vel [>= S, 3] and angular speeds omega [>= S]
    (None: the collider's constant angular speed)."""
    if omega is None:
        omega = torch.full((vel.shape[0],), float(env.colliders[col].omega), dtype=vel.dtype)
    centers, angles = collider_path(env, vel, omega, col)
    return centers, angles, omega


def _motion_at(path, vel, k: int, col: int):
    """Substep k's motion argument of grid_update with collider `col` driven."""
    if path is None:
        return None
    out = [None] * (col + 1)
    out[col] = (path[0][k], vel[k], path[1][k], path[2][k])
    return out


def rollout(env: Env, prm, state, S: int, t0: float = 0.0, keep_all=False, vel=None, omega=None, col: int = 0):
    """Run S substeps; returns the final state (and every state if keep_all).

    ``vel`` [>= S, 3] and ``omega`` [>= S]: per-substep velocities and angular
    speeds (actions) of collider `col`, whose path starts at its configured
    center and angle at the first substep (t0 = 0)."""
    x, v, C, F = state
    states = [state]
    any_oob = False
    path = None
    if vel is not None:
        assert t0 == 0.0 and col < len(env.colliders)
        path = motion_path(env, vel, omega, col)
    for k in range(S):
        motion = _motion_at(path, vel, k, col)
        x, v, C, F, oob = substep(env, prm, x, v, C, F, t0 + k * env.dt, motion)
        any_oob |= oob
        if keep_all:
            states.append((x, v, C, F))
    if keep_all:
        return states, any_oob
    return (x, v, C, F), any_oob


def rollout_vjp(env: Env, prm, state, S: int, cot, t0: float = 0.0, vel=None, omega=None, col: int = 0):
    """Reverse-mode cotangents of the initial state and of the 7 parameters.

    ``cot`` = (x_bar, v_bar, C_bar, F_bar) of the final state (None entries = 0).
    Each substep is re-differentiated from its stored input (per-substep
    checkpointing), so memory stays at one substep's graph. With a collider
    motion ``vel`` it also returns the cotangents of the velocities [S, 3] and
    of the box's starting center [3]: each substep yields those of its own
    (center_k, v_k), and center_k = c0 + dt sum_{j<k} vel_j passes its part to
    every earlier velocity and to c0. With angular speeds ``omega`` as well it
    further returns those of omega [S] and of the starting angle, by the same
    chain through angle_k = angle0 + dt sum_{j<k} omega_j. The actions drive
    collider `col`.
    """
    with torch.no_grad():
        states, _ = rollout(env, prm, state, S, t0, keep_all=True, vel=vel, omega=omega, col=col)
        path = None if vel is None else motion_path(env, vel, omega, col)
    g = [torch.zeros_like(s) if c is None else c.to(DT) for s, c in zip(state, cot)]
    gprm = torch.zeros_like(prm)
    gcen = torch.zeros(S, 3, dtype=DT)
    gvb = torch.zeros(S, 3, dtype=DT)
    gang = torch.zeros(S, dtype=DT)
    gom = torch.zeros(S, dtype=DT)
    for k in reversed(range(S)):
        s_in = [s.detach().clone().requires_grad_(True) for s in states[k]]
        p_in = prm.detach().clone().requires_grad_(True)
        leaves = s_in + [p_in]
        motion = None
        if path is not None:
            mk = tuple(a.detach().clone().requires_grad_(True) for a in (path[0][k], vel[k], path[1][k], path[2][k]))
            leaves = leaves + list(mk)
            motion = [None] * col + [mk]
        with torch.enable_grad():
            out = substep(env, p_in, *s_in, t0 + k * env.dt, motion)[:4]
            grads = torch.autograd.grad(out, leaves, grad_outputs=g, allow_unused=True)
        g = [torch.zeros_like(s) if gr is None else gr for s, gr in zip(s_in, grads[:4])]
        if grads[4] is not None:
            gprm = gprm + grads[4]
        if path is not None:
            for dst, gr in zip((gcen, gvb, gang, gom), grads[5:]):
                if gr is not None:
                    dst[k] = gr
    if vel is None:
        return tuple(g), gprm
    later = torch.flip(torch.cumsum(torch.flip(gcen, [0]), 0), [0]) - gcen   # sum over k > j
    gvel = gvb + env.dt * later
    if omega is None:
        return tuple(g), gprm, gvel, gcen.sum(0)
    later_a = torch.flip(torch.cumsum(torch.flip(gang, [0]), 0), [0]) - gang
    return tuple(g), gprm, gvel, gcen.sum(0), gom + env.dt * later_a, gang.sum()


def rollout_jvp(env: Env, prm, state, S: int, tangent, prm_tangent, t0: float = 0.0, vel=None, vel_tangent=None,
                omega=None, omega_tangent=None):
    """Forward-mode tangent of the final state (dual numbers through the same forward)."""
    import torch.autograd.forward_ad as fwAD
    with torch.no_grad(), fwAD.dual_level():
        st = [fwAD.make_dual(s, ts) for s, ts in zip(state, tangent)]
        p = fwAD.make_dual(prm, prm_tangent)
        path = vv = om = None
        if vel is not None:
            vv = fwAD.make_dual(vel, vel_tangent if vel_tangent is not None else torch.zeros_like(vel))
            if omega is not None:
                om = fwAD.make_dual(omega, omega_tangent if omega_tangent is not None else torch.zeros_like(omega))
            path = motion_path(env, vv, om)
        x, v, C, F = st
        for k in range(S):
            motion = None if path is None else (path[0][k], vv[k], path[1][k], path[2][k])
            x, v, C, F, _ = substep(env, p, x, v, C, F, t0 + k * env.dt, motion)
        return tuple(fwAD.unpack_dual(a).tangent for a in (x, v, C, F))


def param_cotangent_row(gprm) -> np.ndarray:
    """Pack the 7 parameter cotangents into the 8-entry row of the C interface."""
    out = np.zeros(8, dtype=np.float64)
    out[:7] = gprm.detach().numpy()
    return out


def linear_loss_cotangent(weights: np.ndarray, N: int):
    """Cotangents of L = sum_p x_p . w_p: d/dx = w, zero for v, C, F."""
    w = torch.from_numpy(np.asarray(weights, dtype=np.float32)).to(DT)
    return (w, torch.zeros(N, 3, dtype=DT), torch.zeros(N, 3, 3, dtype=DT), torch.zeros(N, 3, 3, dtype=DT))


# ----------------------------------------------------------------------------
# Observation / reward statistics of the manipulation tasks (Appendix E: the
# centre of mass of a subsampled particle set, the variance of its heights,
# mean velocities), as per-env weighted moments
# ----------------------------------------------------------------------------
MOMENT_NAMES = ("w", "x", "y", "z", "xx", "yy", "zz", "xy", "xz", "yz",
                "vx", "vy", "vz", "vxvx", "vyvy", "vzvz", "vxvy", "vxvz", "vyvz")


def moments(x, v, w):
    """Per-env weighted moments [19]: sum w, sum w x (3), sum w x x^T (xx yy zz xy xz yz),
    the same two for v. x, v: [N, 3]; w: [N] weights (0/1 selects a subsample)."""
    x, v, w = (torch.as_tensor(a, dtype=DT) for a in (x, v, w))

    def second(a):
        return torch.stack([(w * a[:, i] * a[:, j]).sum() for i, j in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])

    return torch.cat([w.sum()[None], (w[:, None] * x).sum(0), second(x), (w[:, None] * v).sum(0), second(v)])


def moment_stats(m):
    """Centre of mass, height variance and mean velocity from one env's moments."""
    com = m[1:4] / m[0]
    var_z = m[6] / m[0] - com[2] ** 2
    vbar = m[10:13] / m[0]
    return com, var_z, vbar


# ----------------------------------------------------------------------------
# The flip reward of the HandFlip task (Appendix E): the mean Euclidean distance
# between two mirrored halves of the particles, paired particle by particle,
# and its normalized improvement NI{r} = clamp((r0 - r) / r0, -1, 1) over the
# initial value r0
# ----------------------------------------------------------------------------
def mirror_pairs(x0, axis: int, plane: float):
    """Pairs (lower, upper) of particles mirrored across the plane x[axis] =
    plane in the configuration x0: the particles below the plane, each matched
    to the upper-half particle nearest to its mirror image (a reading: the
    paper names the two halves but not how they are matched). Brute force."""
    x0 = np.asarray(x0, dtype=np.float64)
    low = np.nonzero(x0[:, axis] < plane)[0]
    up = np.nonzero(x0[:, axis] >= plane)[0]
    img = x0[low].copy()
    img[:, axis] = 2.0 * plane - img[:, axis]
    d = ((img[:, None, :] - x0[up][None, :, :]) ** 2).sum(-1)
    return np.stack([low, up[np.argmin(d, axis=1)]], axis=1)


def pair_distance(x, pairs):
    """R_flip = (1 / P) sum_k ||x[a_k] - x[b_k]||_2 over the P pairs (a_k, b_k)."""
    x = torch.as_tensor(x, dtype=DT)
    p = torch.as_tensor(np.ascontiguousarray(pairs), dtype=torch.long)
    if p.numel() == 0:
        return torch.zeros((), dtype=DT)
    return (x[p[:, 0]] - x[p[:, 1]]).norm(dim=1).mean()


def normalized_improvement(r, r0):
    """NI{r} = clamp((r0 - r) / r0, -1, 1)."""
    return torch.clamp((r0 - r) / r0, -1.0, 1.0)
