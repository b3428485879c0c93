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
    mode with the fused G2P + P2G and adjoint-pair schedules."""
    b = Batch(envs, max_substeps=max(S, 1), ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode == "batched-fused":
            from paper_2412_12089_amd import _capi as C
            b.set_option(C.OPT_FUSE, 1)
            b.set_option(C.OPT_FUSE_ADJ, 1)
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
