"""Shared helpers of the GPU parity tests: run a scene through the library
(C interface) and through the FP64 oracle, and compare normwise."""
from __future__ import annotations

import numpy as np
import torch

from oracle import mpm_oracle as O
from paper_2412_12089_amd import scenes
from paper_2412_12089_amd.batch import Batch

STATE_KEYS = ("x", "v", "C", "F")


def relerr(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def particle_maxerr(a, b) -> float:
    """Largest per-particle error relative to the env's rms magnitude:
    max_p ||a_p - b_p|| / sqrt(mean_p ||b_p||^2). A few particles on a wrong
    path pass a normwise check over thousands; they fail this one."""
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    rms = float(np.sqrt(np.mean(np.sum(b * b, axis=1))))
    return float(np.max(np.linalg.norm(a - b, axis=1)) / (rms if rms > 0 else 1.0)) if len(a) else 0.0


# Bars. Normwise per env (the stated ones): x, v 1e-5; C, F 1e-4; gradients
# 1e-3. Per particle (max over particles, relative to the env's rms): ten times
# the normwise bar. Displacement x - x0, normwise: 1e-3, or ten times the FP32
# floor where that is larger. The floor: an FP32 position in [0, 1) is rounded
# at every substep by at most half an ulp (2^-24), an rms of 2^-24 / sqrt(3)
# per step, sqrt(S) times that after S steps; a 10-substep move of ~5e-4 sits
# ~1e-4 above it, so the displacement check is ~100 times tighter on the
# motion than the 1e-5 bar on x, whose magnitude is mostly the starting
# position. (The slow 2 ms dam break moves ~2e-5: there the floor sets the bar.)
TOL_XV, TOL_CF, TOL_GRAD, TOL_DISP, PER_PARTICLE = 1e-5, 1e-4, 1e-3, 1e-3, 10.0
ROUND_RMS = 2.0 ** -24 / np.sqrt(3.0)


def disp_bar(o_x, x0, S) -> float:
    d = np.asarray(o_x, np.float64) - x0
    rms = float(np.sqrt(np.mean(np.sum(d * d, axis=1)))) if len(d) else 0.0
    if S is None or rms == 0.0:
        return TOL_DISP
    return max(TOL_DISP, 10.0 * np.sqrt(3.0 * S) * ROUND_RMS / rms)


def state_errors(g, o, x0):
    """Normwise, per-particle and displacement errors of a state (x, v, C, F)."""
    return dict(x=relerr(g[0], o[0]), v=relerr(g[1], o[1]), C=relerr(g[2], o[2]), F=relerr(g[3], o[3]),
                x_p=particle_maxerr(g[0], o[0]), v_p=particle_maxerr(g[1], o[1]),
                C_p=particle_maxerr(g[2], o[2]), F_p=particle_maxerr(g[3], o[3]),
                dx=relerr(np.asarray(g[0], np.float64) - x0, np.asarray(o[0], np.float64) - x0))


def assert_state(g, o, x0, tag, announce=print, tol_xv=TOL_XV, tol_cf=TOL_CF, S=None):
    """S: substeps of the rollout (sets the displacement floor), None = 1e-3 bar."""
    x0 = np.asarray(x0, np.float64)
    e = state_errors(g, o, x0)
    bar = disp_bar(o[0], x0, S)
    announce(f"{tag}: x {e['x']:.2e} v {e['v']:.2e} C {e['C']:.2e} F {e['F']:.2e} | per particle x {e['x_p']:.2e} "
             f"v {e['v_p']:.2e} C {e['C_p']:.2e} F {e['F_p']:.2e} | displacement {e['dx']:.2e} (bar {bar:.1e})")
    assert e["x"] < tol_xv and e["v"] < tol_xv, (tag, e)
    assert e["C"] < tol_cf and e["F"] < tol_cf, (tag, e)
    assert e["x_p"] < PER_PARTICLE * tol_xv and e["v_p"] < PER_PARTICLE * tol_xv, (tag, e)
    assert e["C_p"] < PER_PARTICLE * tol_cf and e["F_p"] < PER_PARTICLE * tol_cf, (tag, e)
    assert e["dx"] < bar, (tag, e, bar)
    return e


def assert_grads(g, o, tag, announce=print, skip=()):
    n = [relerr(a, b) for a, b in zip(g, o)]
    m = [particle_maxerr(a, b) for a, b in zip(g, o)]
    announce(f"{tag}: grad x {n[0]:.2e} v {n[1]:.2e} C {n[2]:.2e} F {n[3]:.2e} | per particle x {m[0]:.2e} "
             f"v {m[1]:.2e} C {m[2]:.2e} F {m[3]:.2e}")
    for i in range(4):
        if i in skip:
            continue
        assert n[i] < TOL_GRAD and m[i] < PER_PARTICLE * TOL_GRAD, (tag, i, n[i], m[i])


def assert_params(gp, op, idx, tag, prm, announce=print, tol=TOL_GRAD):
    """Parameter cotangents (E, nu, rho, Vp, sigma_y, K, gamma) against the
    oracle's. prm: the env's parameter row. The Vp cotangent is exactly 0 on the
    GPU (Vp cancels between particle mass and force) and at rounding level in
    the oracle, measured against |E dL/dE| + |sigma_y dL/dsigma_y| + |K dL/dK|."""
    from oracle import mpm_oracle as O
    p = np.asarray(prm, dtype=np.float64)
    scale = abs(p[0] * op[0]) + abs(p[4] * op[4]) + abs(p[5] * op[5])
    for k in idx:
        if k == 3:
            announce(f"{tag}: dparam[Vp] gpu {gp[3]:.3e} oracle {op[3]:.3e} (Vp dL/dVp vs {scale:.3e})")
            assert gp[3] == 0.0 and abs(p[3] * op[3]) <= 1e-9 * scale, (tag, gp[3], op[3])
            continue
        if op[k] == 0.0:   # e.g. no particle yielded: the sigma_y cotangent is exactly zero
            announce(f"{tag}: dparam[{O.PARAM_NAMES[k]}] gpu {gp[k]:.6e} vs exact 0")
            assert gp[k] == 0.0, (tag, k, gp[k])
            continue
        e = abs(gp[k] - op[k]) / abs(op[k])
        announce(f"{tag}: dparam[{O.PARAM_NAMES[k]}] gpu {gp[k]:.6e} oracle {op[k]:.6e} rel {e:.2e}")
        assert e < tol, (tag, k, gp[k], op[k])


def to_np(t) -> np.ndarray:
    return t.detach().cpu().double().numpy()


def env_slices(envs):
    off = np.concatenate([[0], np.cumsum([e.n_particles for e in envs])]).astype(int)
    return [slice(off[i], off[i + 1]) for i in range(len(envs))]


def random_cotangents(envs, seed=123, scale=(1.0, 1.0, 0.01, 1.0)):
    """Seeded float32 cotangents of the final (x, v, C, F) for each env."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for e in envs:
        N = e.n_particles
        out.append(tuple(np.float32(s) * rng.standard_normal(shape).astype(np.float32)
                         for s, shape in zip(scale, ((N, 3), (N, 3), (N, 3, 3), (N, 3, 3)))))
    return out


def gpu_rollout(envs, S, K, mode="batched", cots=None, timing=False):
    """Forward S substeps (recorded) and, if cots are given, the backward.

    Returns dict(state=(x,v,C,F) numpy float64, grads=(dx,dv,dC,dF) or None,
    dparams=[E,8] or None, status=sync code). mode "batched-fused": the batched
    mode with the fused G2P + P2G and adjoint-pair schedules; "batched-pull":
    the pull scatters with both fusions and the flagged-tile list."""
    from paper_2412_12089_amd import _capi as C
    b = Batch(envs, max_substeps=max(S, 1), ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode in ("batched-fused", "batched-pull"):
            b.set_option(C.OPT_FUSE, 1)
            b.set_option(C.OPT_FUSE_ADJ, 1)
        if mode == "batched-pull":
            for opt, val in ((C.OPT_P2G, 3), (C.OPT_G2P_ADJ, 3), (C.OPT_GRID_LIST, 1)):
                b.set_option(opt, val)
        b.set_particles_from_specs()
        b.forward(S, record=cots is not None)
        st = tuple(to_np(t) for t in b.get_particles())
        grads = dparams = None
        if cots is not None:
            cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
            dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
            grads = tuple(to_np(t) for t in (dx, dv, dC, dF))
            dparams = to_np(dp)
        status = b.sync(raise_on_error=False)
        return dict(state=st, grads=grads, dparams=dparams, status=status, errors=b.env_errors())
    finally:
        b.close()


def oracle_rollout(spec, S, cot=None):
    env, prm, st = O.env_from_spec(spec)
    (x, v, C, F), oob = O.rollout(env, prm, st, S)
    out = dict(state=tuple(t.numpy() for t in (x, v, C, F)), oob=oob)
    if cot is not None:
        c = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).double() for a in cot)
        g, gp = O.rollout_vjp(env, prm, st, S, c)
        out["grads"] = tuple(t.numpy() for t in g)
        out["dparams"] = O.param_cotangent_row(gp)
    return out


def make_env(material, N=3000, n=32, seed=0, dt=1e-4, lo=0.35, side=0.22, v_scale=0.5, F_dev=0.0,
             E=5e3, nu=0.3, sigma_y=50.0, K=1e4, gamma=7.0, collider=None, gravity=scenes.GRAVITY):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = scenes._f32(lo + rng.uniform(0, side, size=(N, 3)))
    v = scenes._f32(rng.uniform(-v_scale, v_scale, size=(N, 3)))
    Cm = np.zeros((N, 3, 3), dtype=np.float32)
    dev = np.full((N, 1, 1), F_dev[0] if isinstance(F_dev, tuple) else F_dev)
    if isinstance(F_dev, tuple):      # alternate two deviation scales between particles
        dev[1::2] = F_dev[1]
    F = np.broadcast_to(np.eye(3), (N, 3, 3)) + dev * rng.standard_normal((N, 3, 3))
    if material in (scenes.FLUID_TAIT, scenes.FLUID_PAPER):
        F = np.cbrt(np.linalg.det(F))[:, None, None] * np.eye(3)
    F = scenes._f32(F)
    return scenes.EnvSpec(n=n, dt=dt, material=material, E=E, nu=nu, rho=1e3, Vp=side ** 3 / N,
                          sigma_y=sigma_y, K=K, gamma=gamma, collider=collider, gravity=gravity,
                          x=x, v=v, C=Cm, F=F)
