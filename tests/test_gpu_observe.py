"""Device-side observation / reward moments and their VJP against the FP64
oracle, and the chain rollout -> moments -> task statistics -> loss through
both autograd Functions."""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import make_env, relerr
from oracle import mpm_oracle as O
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def announce(msg):
    print(f"[gpu-observe] {msg}", flush=True)


def envs3():
    return [make_env(scenes.NEOHOOKEAN, N=1500, seed=70), make_env(scenes.COROTATED, N=777, seed=71, E=1e4, nu=0.25),
            make_env(scenes.FLUID_TAIT, N=2600, n=48, seed=72)]


@pytest.mark.parametrize("stride", [1, 5])
def test_moments_and_vjp_match_oracle(stride):
    from paper_2412_12089_amd.batch import Batch
    from paper_2412_12089_amd import observe
    envs = envs3()
    dev = torch.device("cuda:0")
    b = Batch(envs, max_substeps=4, ckpt_every=2)
    try:
        rng = np.random.default_rng(73)
        N = b.N
        x = torch.from_numpy(rng.uniform(0.2, 0.8, size=(N, 3)).astype(np.float32)).to(dev)
        v = torch.from_numpy(rng.standard_normal((N, 3)).astype(np.float32)).to(dev)
        w = observe.subsample_weights(b, stride) if stride > 1 else None
        m = b.moments(x, v, w).cpu().numpy()
        g = torch.from_numpy(rng.standard_normal((len(envs), 20)))
        g[:, 19] = 0.0
        gx, gv = b.moments_vjp(x, v, w, g.to(dev))
        gx, gv = gx.cpu().numpy(), gv.cpu().numpy()
        b.sync()
    finally:
        b.close()
    xs, vs = x.cpu().double(), v.cpu().double()
    ws = torch.ones(N, dtype=torch.float64) if w is None else w.cpu().double()
    for i, (lo, hi) in enumerate(zip(b.offsets[:-1], b.offsets[1:])):
        xi = xs[lo:hi].clone().requires_grad_(True)
        vi = vs[lo:hi].clone().requires_grad_(True)
        mo = O.moments(xi, vi, ws[lo:hi])
        err = relerr(m[i, :19], mo.detach().numpy())
        (mo * g[i, :19]).sum().backward()
        ex, ev = relerr(gx[lo:hi], xi.grad.numpy()), relerr(gv[lo:hi], vi.grad.numpy())
        announce(f"stride {stride} env {i}: moments {err:.2e}, vjp x {ex:.2e} v {ev:.2e}")
        assert err < 1e-6 and ex < 1e-5 and ev < 1e-5
        assert m[i, 19] == 0.0


def test_rollout_to_task_statistics_chain():
    # loss = height variance + CoM x of a subsample at the end of a rollout, per env;
    # its gradient w.r.t. the initial state through both Functions vs the oracle
    from paper_2412_12089_amd.batch import Batch, rollout
    from paper_2412_12089_amd import observe
    envs = envs3()[:2]
    S, K = 5, 2
    dev = torch.device("cuda:0")
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in envs], axis=0)).to(dev)
    st = [cat(k).requires_grad_(True) for k in ("x", "v", "C", "F")]
    params = torch.tensor(np.stack([e.params() for e in envs]), dtype=torch.float64, requires_grad=True)
    b = Batch(envs, max_substeps=S, ckpt_every=K)
    try:
        w = observe.subsample_weights(b, 3)
        xs, vs, _, _ = rollout(b, S, *st, params)
        m = observe.moments(b, xs, vs, w)
        loss = (observe.height_variance(m) + observe.center_of_mass(m)[:, 0] + observe.mean_velocity(m)[:, 2]).sum()
        loss.backward()
        wn = w.cpu().double()
    finally:
        b.close()
    for i, (lo, hi) in enumerate(zip(b.offsets[:-1], b.offsets[1:])):
        env, prm, s0 = O.env_from_spec(envs[i])
        (xf, vf, _, _), _ = O.rollout(env, prm, s0, S)
        xf = xf.clone().requires_grad_(True)
        vf = vf.clone().requires_grad_(True)
        com, var_z, vbar = O.moment_stats(O.moments(xf, vf, wn[lo:hi]))
        (var_z + com[0] + vbar[2]).backward()
        g, _ = O.rollout_vjp(env, prm, s0, S, (xf.grad, vf.grad, None, None))
        errs = [relerr(t.grad[lo:hi].cpu().double().numpy(), og.numpy()) for t, og in zip(st, g)]
        announce(f"env {i}: chain grads x {errs[0]:.2e} v {errs[1]:.2e} C {errs[2]:.2e} F {errs[3]:.2e}")
        assert max(errs) < 1e-3


def test_flip_distance_and_vjp_match_oracle():
    # the HandFlip flip term on mirrored pairs plus random pairs and pairs out of range (skipped)
    from paper_2412_12089_amd.batch import Batch
    from paper_2412_12089_amd import observe
    envs = envs3()
    dev = torch.device("cuda:0")
    b = Batch(envs, max_substeps=2, ckpt_every=2)
    try:
        rng = np.random.default_rng(74)
        N = b.N
        x = torch.from_numpy(rng.uniform(0.2, 0.8, size=(N, 3)).astype(np.float32)).to(dev)
        pm = observe.mirror_pairs(b.counts, x, axis=2)
        pr = np.stack([np.repeat(np.arange(3), 50), rng.integers(0, 700, 150), rng.integers(0, 700, 150)], 1)
        bad = np.array([[5, 0, 1], [0, -1, 2], [1, 0, 10 ** 6]])
        pairs = torch.cat([pm, torch.from_numpy(pr.astype(np.int32)), torch.from_numpy(bad.astype(np.int32))])
        out = b.pair_distance(x, pairs).cpu().numpy()
        g = torch.from_numpy(rng.standard_normal(3))
        gx = b.pair_distance_vjp(x, pairs, torch.from_numpy(out).to(dev), g.to(dev)).cpu().numpy()
        b.sync()
    finally:
        b.close()
    xs = x.cpu().double()
    P = pairs.numpy()
    for i, (lo, hi) in enumerate(zip(b.offsets[:-1], b.offsets[1:])):
        mine = P[(P[:, 0] == i) & (P[:, 1] >= 0) & (P[:, 2] >= 0) & (P[:, 1] < hi - lo) & (P[:, 2] < hi - lo)][:, 1:]
        xi = xs[lo:hi].clone().requires_grad_(True)
        r = O.pair_distance(xi, mine)
        (r * float(g[i])).backward()
        er = abs(out[i, 0] - float(r)) / float(r)
        eg = relerr(gx[lo:hi], xi.grad.numpy())
        announce(f"env {i}: {len(mine)} pairs, flip distance {out[i, 0]:.6f} rel {er:.2e}, vjp {eg:.2e}")
        assert out[i, 1] == len(mine) and er < 1e-6 and eg < 1e-5


def test_rollout_to_flip_reward_chain():
    # reward = NI of the flip distance at the end of a rollout against its initial value; its gradient
    # w.r.t. the initial state through the rollout and the flip-distance Functions vs the oracle
    from paper_2412_12089_amd.batch import Batch, rollout
    from paper_2412_12089_amd import observe
    envs = envs3()[:2]
    S, K = 5, 2
    dev = torch.device("cuda:0")
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in envs], axis=0)).to(dev)
    st = [cat(k).requires_grad_(True) for k in ("x", "v", "C", "F")]
    params = torch.tensor(np.stack([e.params() for e in envs]), dtype=torch.float64, requires_grad=True)
    b = Batch(envs, max_substeps=S, ckpt_every=K)
    try:
        pairs = observe.mirror_pairs(b.counts, st[0].detach(), axis=2)
        r0 = observe.flip_distance(b, st[0].detach(), pairs)
        xs, _, _, _ = rollout(b, S, *st, params)
        reward = observe.normalized_improvement(observe.flip_distance(b, xs, pairs), r0)
        reward.sum().backward()
    finally:
        b.close()
    P = pairs.numpy()
    for i, (lo, hi) in enumerate(zip(b.offsets[:-1], b.offsets[1:])):
        env, prm, s0 = O.env_from_spec(envs[i])
        mine = P[P[:, 0] == i][:, 1:]
        (xf, _, _, _), _ = O.rollout(env, prm, s0, S)
        xf = xf.clone().requires_grad_(True)
        O.normalized_improvement(O.pair_distance(xf, mine), O.pair_distance(s0[0], mine)).backward()
        g, _ = O.rollout_vjp(env, prm, s0, S, (xf.grad, None, None, None))
        errs = [relerr(t.grad[lo:hi].cpu().double().numpy(), og.numpy()) for t, og in zip(st, g)]
        announce(f"env {i}: flip reward chain grads x {errs[0]:.2e} v {errs[1]:.2e} C {errs[2]:.2e} F {errs[3]:.2e}")
        assert max(errs) < 1e-3
