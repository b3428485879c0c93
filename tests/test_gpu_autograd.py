"""The torch.autograd.Function over the library (forward records, backward runs
the hand-written adjoint): gradients of the initial state, the material
parameters and the collider actions against the FP64 oracle, and directional
derivatives against central differences of the GPU forward."""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import make_env, relerr
from oracle import mpm_oracle as O
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

BOX = scenes.BoxCollider(center=(0.62, 0.46, 0.46), half=(0.04, 0.2, 0.2), velocity=(-0.5, 0.0, 0.0),
                         alpha=64.0, mu_b=0.5)
S, K = 6, 3


def announce(msg):
    print(f"[gpu-autograd] {msg}", flush=True)


def setup():
    envs = [make_env(scenes.NEOHOOKEAN, N=1500, seed=60, F_dev=0.02),
            make_env(scenes.FLUID_TAIT, N=2000, seed=61, collider=BOX, v_scale=0.2)]
    rng = np.random.default_rng(62)
    N = sum(e.n_particles for e in envs)
    wx = rng.standard_normal((N, 3)).astype(np.float32)
    wv = rng.standard_normal((N, 3)).astype(np.float32)
    actions = (np.array(BOX.velocity) + 0.3 * rng.standard_normal((2, S, 3))).astype(np.float32)
    return envs, wx, wv, actions


def inputs(envs, actions, dev, grad=True):
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in envs], axis=0)).to(dev)
    st = [cat(k).requires_grad_(grad) for k in ("x", "v", "C", "F")]
    params = torch.tensor(np.stack([e.params() for e in envs]), dtype=torch.float64, requires_grad=grad)
    act = torch.from_numpy(actions).requires_grad_(grad)
    return st, params, act


def loss_of(out, wx, wv):
    return (out[0] * wx).sum() + (out[1] * wv).sum()


def test_autograd_function_matches_oracle():
    from paper_2412_12089_amd.batch import Batch, rollout
    dev = torch.device("cuda:0")
    envs, wx, wv, actions = setup()
    st, params, act = inputs(envs, actions, dev)
    batch = Batch(envs, max_substeps=S, ckpt_every=K)
    try:
        out = rollout(batch, S, *st, params, act)
        loss = loss_of(out, torch.from_numpy(wx).to(dev), torch.from_numpy(wv).to(dev))
        # re-use the batch before the backward: the Function must re-run its own forward
        batch.set_particles_from_specs()
        batch.forward(2)
        loss.backward()
    finally:
        batch.close()
    offs = np.cumsum([0] + [e.n_particles for e in envs])
    for i, e in enumerate(envs):
        sl = slice(offs[i], offs[i + 1])
        env, prm, st0 = O.env_from_spec(e)
        cot = (torch.from_numpy(wx[sl]).double(), torch.from_numpy(wv[sl]).double(), None, None)
        if e.collider is not None:
            g, gp, gvel, _ = O.rollout_vjp(env, prm, st0, S, cot, vel=torch.from_numpy(actions[i]).double())
            ea = relerr(act.grad[i].numpy(), gvel.numpy())
            announce(f"env {i}: actions rel {ea:.2e}")
            assert ea < 1e-3
        else:
            g, gp = O.rollout_vjp(env, prm, st0, S, cot)
            assert np.all(act.grad[i].numpy() == 0.0)
        errs = [relerr(t.grad[sl].cpu().double().numpy(), og.numpy()) for t, og in zip(st, g)]
        announce(f"env {i}: grad x {errs[0]:.2e} v {errs[1]:.2e} C {errs[2]:.2e} F {errs[3]:.2e}")
        assert max(errs) < 1e-3
        row = O.param_cotangent_row(gp)
        for k in ([0, 1] if e.material == scenes.NEOHOOKEAN else [5, 6]):
            r = abs(params.grad[i, k].item() - row[k]) / abs(row[k])
            announce(f"env {i}: dparam[{k}] rel {r:.2e}")
            assert r < 1e-3


def test_autograd_function_matches_central_differences():
    from paper_2412_12089_amd.batch import Batch, rollout
    dev = torch.device("cuda:0")
    envs, wx, wv, actions = setup()
    wxt, wvt = torch.from_numpy(wx).to(dev), torch.from_numpy(wv).to(dev)
    st, params, act = inputs(envs, actions, dev)
    batch = Batch(envs, max_substeps=S, ckpt_every=K)
    try:
        loss = loss_of(rollout(batch, S, *st, params, act), wxt, wvt)
        loss.backward()
        rng = np.random.default_rng(63)
        dv = torch.from_numpy(rng.standard_normal(tuple(st[1].shape)).astype(np.float32)).to(dev)
        da = torch.from_numpy(rng.standard_normal(actions.shape).astype(np.float32))

        def value(vv, aa):
            with torch.no_grad():
                s2, p2, a2 = inputs(envs, aa.numpy(), dev, grad=False)
                out = rollout(batch, S, s2[0], vv, s2[2], s2[3], p2, a2)
                return loss_of(out, wxt, wvt).double().item()

        v0 = st[1].detach()
        a0 = torch.from_numpy(actions)
        for name, h, plus, minus, an in (
                ("v", 1e-3, lambda h: value(v0 + h * dv, a0), lambda h: value(v0 - h * dv, a0),
                 (st[1].grad * dv).sum().item()),
                ("actions", 1e-3, lambda h: value(v0, a0 + h * da), lambda h: value(v0, a0 - h * da),
                 (act.grad * da).sum().item())):
            fd = (plus(h) - minus(h)) / (2 * h)
            announce(f"{name}: central difference {fd:.6e} vs adjoint {an:.6e}")
            assert abs(fd - an) <= 1e-2 * abs(an)
    finally:
        batch.close()


def test_autograd_drives_several_colliders():
    # actions [E, K, S, 3] and spins [E, K, S] on a gripper's first two slots (a jaw and a finger) through the
    # autograd Function: each slot's action cotangents against the oracle with that slot driven alone (the
    # other slot keeps its constant motion in both)
    import dataclasses
    from test_gpu_parity import GRIP
    from paper_2412_12089_amd.batch import Batch, rollout
    dev = torch.device("cuda:0")
    spec = make_env(scenes.FLUID_TAIT, N=2500, seed=70, collider=GRIP[0], v_scale=0.2)
    spec = dataclasses.replace(spec, more_colliders=GRIP[1:])
    rng = np.random.default_rng(71)
    wx = rng.standard_normal((spec.n_particles, 3)).astype(np.float32)
    wxt = torch.from_numpy(wx).to(dev)
    for slot in (0, 1):
        col = GRIP[slot]
        vel = (np.array(col.velocity) + 0.3 * rng.standard_normal((S, 3))).astype(np.float32)
        om = (col.omega + 2.0 * rng.standard_normal(S)).astype(np.float32)
        act = np.zeros((1, 2, S, 3), np.float32)
        spn = np.zeros((1, 2, S), np.float32)
        for k in (0, 1):   # the other slot moves at its constant velocity and spin
            act[0, k] = GRIP[k].velocity
            spn[0, k] = GRIP[k].omega
        act[0, slot], spn[0, slot] = vel, om
        st = [torch.from_numpy(np.asarray(a, np.float32)).to(dev).requires_grad_(True) for a in (spec.x, spec.v, spec.C, spec.F)]
        params = torch.from_numpy(spec.params()[None]).to(dev).requires_grad_(True)
        at = torch.from_numpy(act).to(dev).requires_grad_(True)
        sp = torch.from_numpy(spn).to(dev).requires_grad_(True)
        batch = Batch([spec], max_substeps=S, ckpt_every=K)
        try:
            out = rollout(batch, S, *st, params, at, None, sp)
            (out[0] * wxt).sum().backward()
        finally:
            batch.close()
        env, prm, st0 = O.env_from_spec(spec)
        cot = (torch.from_numpy(wx).double(), None, None, None)
        _, _, gvel, _, gom, _ = O.rollout_vjp(env, prm, st0, S, cot, vel=torch.from_numpy(vel).double(),
                                               omega=torch.from_numpy(om).double(), col=slot)
        ea = relerr(at.grad[0, slot].cpu().numpy(), gvel.numpy())
        es = relerr(sp.grad[0, slot].cpu().numpy(), gom.numpy())
        announce(f"slot {slot} driven: actions rel {ea:.2e}, spins rel {es:.2e}")
        assert ea < 1e-3 and es < 1e-3
