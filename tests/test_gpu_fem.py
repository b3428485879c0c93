"""The FEM path (include/mpm_fem.h) against the FP64 FEM oracle: forward
states, the reverse-mode cotangents of the initial state, of every
substep's activations and of the parameters, the autograd Function, and the
interface's edge cases."""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import particle_maxerr, relerr
from oracle import fem_oracle as FO
from paper_2412_12089_amd import _capi as C
from paper_2412_12089_amd import fem_scenes as FS

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

# Bars (FP32 library vs FP64 oracle), normwise per env: the displacement x - x0
# and v 1e-4; every cotangent 1e-3 (the MPM gradient bar); per node, ten
# times these relative to the env's rms.
TOL_STATE, TOL_GRAD, PER_NODE = 1e-4, 1e-3, 10.0


def announce(msg):
    print(f"[gpu-fem] {msg}", flush=True)


def make_batch(w, max_substeps=None):
    from paper_2412_12089_amd.fem import FemBatch
    dev = torch.device("cuda:0")
    b = FemBatch(w.tets, w.n_envs, w.X.shape[1], w.substeps if max_substeps is None else max_substeps, w.dt,
                 w.gravity, dev)
    b.set_rest(torch.from_numpy(w.X).to(dev))
    b.set_params(w.params)
    return b


def run_gpu(w, envs_for_grad=True, seed=0):
    dev = torch.device("cuda:0")
    b = make_batch(w)
    rng = np.random.default_rng(seed)
    gx = rng.standard_normal(w.x0.shape).astype(np.float32)
    gv = (1e-2 * rng.standard_normal(w.x0.shape)).astype(np.float32)
    b.set_state(torch.from_numpy(w.x0).to(dev), torch.from_numpy(w.v0).to(dev))
    b.forward(w.substeps, torch.from_numpy(w.act).to(dev), record=True)
    x, v = b.get_state()
    dx, dv, da, dp = b.backward(torch.from_numpy(gx).to(dev), torch.from_numpy(gv).to(dev))
    assert b.sync(raise_on_error=False) == C.MPM_OK
    out = [t.cpu().numpy() for t in (x, v, dx, dv, da, dp)]
    b.close()
    return out, gx, gv


def oracle_env(w, e, gx, gv):
    mesh = FO.Mesh(w.tets)
    x, v = FO.rollout(mesh, w.X[e], w.params[e], w.x0[e], w.v0[e], w.act[:, e], w.substeps, w.dt)
    g = FO.rollout_vjp(mesh, w.X[e], w.params[e], w.x0[e], w.v0[e], w.act[:, e], w.substeps, w.dt, gx[e], gv[e])
    return [t.numpy() for t in (x, v)], [t.numpy() for t in g]


def check_env(tag, w, e, gpu, o, og):
    x, v, dx, dv, da, dp = gpu
    x0 = w.x0[e].astype(np.float64)
    errs = dict(disp=relerr(x[e] - x0, o[0] - x0), v=relerr(v[e], o[1]),
                disp_n=particle_maxerr(x[e] - x0, o[0] - x0), v_n=particle_maxerr(v[e], o[1]),
                dx=relerr(dx[e], og[0]), dv=relerr(dv[e], og[1]), dact=relerr(da[:, e], og[2]),
                dx_n=particle_maxerr(dx[e], og[0]), dv_n=particle_maxerr(dv[e], og[1]))
    announce(f"{tag} env {e}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for k in ("disp", "v"):
        assert errs[k] < TOL_STATE, (tag, e, k, errs[k])
        assert errs[k + "_n"] < PER_NODE * TOL_STATE, (tag, e, k, errs[k + "_n"])
    for k in ("dx", "dv", "dact"):
        assert errs[k] < TOL_GRAD, (tag, e, k, errs[k])
    for k in ("dx", "dv"):
        assert errs[k + "_n"] < PER_NODE * TOL_GRAD, (tag, e, k, errs[k + "_n"])
    # parameters: relative per component where the oracle's value is above its noise
    ref = og[3]
    scale = np.abs(ref * np.maximum(np.abs(w.params[e]), 1e-3)).max()
    for c, name in enumerate(FO.FEM_PARAMS):
        if abs(ref[c] * max(abs(w.params[e][c]), 1e-3)) < 1e-6 * scale:
            continue
        rel = abs(dp[e][c] - ref[c]) / abs(ref[c])
        assert rel < TOL_GRAD, (tag, e, name, dp[e][c], ref[c])


@pytest.mark.parametrize("seed", [3, 4])
def test_small_mesh_forward_and_backward_match_oracle(seed):
    """12 nodes, 12 elements (one per thread), three envs with their own
    parameters, half of them pressing into the ground."""
    w = FS.two_cubes(seed=seed, n_envs=3, substeps=12)
    announce(f"two_cubes seed {seed}: E {w.n_envs} n {w.X.shape[1]} T {w.tets.shape[0]} S {w.substeps}")
    gpu, gx, gv = run_gpu(w, seed=seed)
    for e in range(w.n_envs):
        o, og = oracle_env(w, e, gx, gv)
        check_env("two_cubes", w, e, gpu, o, og)


def test_jumper_full_size_matches_oracle():
    """The jumper at its full size (199 nodes, 480 elements: two per thread)
    over one 80-substep frame, on two of four envs."""
    w = FS.soft_jumper(seed=11, n_envs=4, substeps=80)
    announce(f"jumper: E {w.n_envs} n {w.X.shape[1]} T {w.tets.shape[0]} S {w.substeps}")
    gpu, gx, gv = run_gpu(w, seed=5)
    for e in (0, 3):
        o, og = oracle_env(w, e, gx, gv)
        check_env("jumper", w, e, gpu, o, og)


def test_bench_size_sampled_envs_match_oracle():
    """The bench's FEM configuration (4096 jumpers, one 80-substep frame, the
    same seed), forward and backward in one launch each; envs at both ends of
    the batch against the oracle."""
    w = FS.soft_jumper(seed=7, n_envs=4096, substeps=80)
    announce(f"bench size: E {w.n_envs} n {w.X.shape[1]} T {w.tets.shape[0]} S {w.substeps}")
    gpu, gx, gv = run_gpu(w, seed=6)
    for e in (0, 4095):
        o, og = oracle_env(w, e, gx, gv)
        check_env("bench-size", w, e, gpu, o, og)


def test_large_mesh_four_elements_per_thread():
    """A 4 x 4 x 6 block of cubes (175 nodes, 576 elements: the launch with
    four per thread), stretched and moving, standing on the ground."""
    rng = np.random.default_rng(21)
    Xm, tets = FS.cube_lattice_mesh([(i, j, k) for i in range(4) for j in range(4) for k in range(6)], 0.02)
    E, S, n, T = 2, 10, Xm.shape[0], tets.shape[0]
    X = np.stack([Xm + [0.1 * e, 0.0, 0.0] for e in range(E)]).astype(np.float32)
    x0 = (X * np.array([1.02, 0.99, 1.0])).astype(np.float32)
    x0[:, :, 2] -= 0.0005
    v0 = (0.2 * rng.standard_normal((E, n, 3))).astype(np.float32)
    prm = np.tile([800.0, 1200.0, 1.0, 0.5, 200.0, 0.05, 0.05, 0.0], (E, 1))
    act = rng.uniform(-0.2, 0.2, size=(S, E, T)).astype(np.float32)
    w = FS.FemWorkload("block", tets, X, x0, v0, prm, act, 1e-4, S)
    announce(f"block: E {E} n {n} T {T} S {S}")
    gpu, gx, gv = run_gpu(w, seed=7)
    for e in range(E):
        o, og = oracle_env(w, e, gx, gv)
        check_env("block", w, e, gpu, o, og)


def test_mesh_whose_adjoint_needs_more_than_64_kib_of_lds():
    """960 elements on 270 nodes: the adjoint block holds 68 KB of LDS (the
    launch raises the kernel's dynamic-LDS limit) and four elements per thread."""
    rng = np.random.default_rng(31)
    Xm, tets = FS.cube_lattice_mesh([(i, j, k) for i in range(4) for j in range(5) for k in range(8)], 0.02)
    E, S, n, T = 2, 6, Xm.shape[0], tets.shape[0]
    assert (n, T) == (270, 960)
    X = np.stack([Xm + [0.2 * e, 0.0, 0.01] for e in range(E)]).astype(np.float32)
    x0 = (X + 0.0004 * rng.standard_normal(X.shape)).astype(np.float32)
    v0 = (0.1 * rng.standard_normal((E, n, 3))).astype(np.float32)
    prm = np.tile([900.0, 1100.0, 1.0, 0.3, 150.0, 0.05, 0.05, 0.0], (E, 1))
    act = rng.uniform(-0.15, 0.15, size=(S, E, T)).astype(np.float32)
    w = FS.FemWorkload("big_block", tets, X, x0, v0, prm, act, 1e-4, S)
    announce(f"big block: E {E} n {n} T {T} S {S}")
    gpu, gx, gv = run_gpu(w, seed=8)
    for e in range(E):
        o, og = oracle_env(w, e, gx, gv)
        check_env("big_block", w, e, gpu, o, og)


def test_chained_rollouts_match_one_rollout():
    """Two env steps through one batch in one autograd graph (the first step's
    backward re-runs its forward, its record having been replaced) against one
    rollout over both: the same states, and the same gradients of the initial
    state, the activations and the parameters."""
    from paper_2412_12089_amd.fem import rollout
    dev = torch.device("cuda:0")
    w = FS.two_cubes(seed=9, n_envs=3, substeps=12)
    b = make_batch(w)
    S1 = 5

    def leaves():
        return (torch.from_numpy(w.x0).to(dev).requires_grad_(True), torch.from_numpy(w.v0).to(dev).requires_grad_(True),
                torch.from_numpy(w.act).to(dev).requires_grad_(True), torch.from_numpy(w.params).requires_grad_(True))

    x0, v0, act, prm = leaves()
    x1, v1 = rollout(b, S1, x0, v0, act[:S1], prm)
    x2, v2 = rollout(b, w.substeps - S1, x1, v1, act[S1:], prm)
    ((x2 - x2.detach().mean()) ** 2).sum().backward()
    g_chain = [t.grad.clone() for t in (x0, v0, act, prm)]
    r0, rv0, ra, rp = leaves()
    xa, va = rollout(b, w.substeps, r0, rv0, ra, rp)
    ((xa - xa.detach().mean()) ** 2).sum().backward()
    assert torch.equal(x2, xa) and torch.equal(v2, va)
    for name, g, r in zip(("x0", "v0", "act", "params"), g_chain, (r0.grad, rv0.grad, ra.grad, rp.grad)):
        assert torch.allclose(g, r, rtol=1e-5, atol=1e-6 * float(r.abs().max())), name
    b.close()


def test_zero_substeps_and_missing_activations():
    dev = torch.device("cuda:0")
    w = FS.two_cubes(seed=5, n_envs=2, substeps=4)
    b = make_batch(w)
    x0, v0 = torch.from_numpy(w.x0).to(dev), torch.from_numpy(w.v0).to(dev)
    # S = 0: the state is unchanged and the backward is the identity with zero parameter cotangents
    b.set_state(x0, v0)
    b.forward(0, None, record=True)
    x, v = b.get_state()
    assert torch.equal(x, x0) and torch.equal(v, v0)
    gx = torch.randn_like(x0)
    dx, dv, da, dp = b.backward(gx, None)
    assert torch.equal(dx, gx) and torch.count_nonzero(dv) == 0 and da.numel() == 0
    assert torch.count_nonzero(dp) == 0
    # act = None is all-zero activations
    b.set_state(x0, v0)
    b.forward(4, None)
    xa, va = b.get_state()
    b.set_state(x0, v0)
    b.forward(4, torch.zeros(4, w.n_envs, w.tets.shape[0], device=dev))
    xb, vb = b.get_state()
    assert torch.equal(xa, xb) and torch.equal(va, vb)
    b.close()


def test_interface_errors():
    dev = torch.device("cuda:0")
    w = FS.two_cubes(seed=6, n_envs=2, substeps=4)
    b = make_batch(w, max_substeps=4)
    b.set_state(torch.from_numpy(w.x0).to(dev))
    dx = torch.empty(w.n_envs, w.X.shape[1], 3, device=dev)
    dv = torch.empty_like(dx)
    assert b.lib.mpm_fem_backward(b.h, None, None, C.ptr(dx), C.ptr(dv), None, None) == C.MPM_BAD_STATE
    assert b.lib.mpm_fem_forward(b.h, -1, None, 0) == C.MPM_INVALID_ARG
    with pytest.raises(C.MPMError) as ei:
        b.forward(5, None, record=True)   # longer than the tape
    assert ei.value.code == C.MPM_BAD_STATE
    bad = w.params.copy()
    bad[1, 1] = -1.0
    with pytest.raises(C.MPMError) as ei:
        b.set_params(bad)
    assert ei.value.code == C.MPM_INVALID_ARG
    # a degenerate rest shape is refused and the previous rest data kept
    b.set_state(torch.from_numpy(w.x0).to(dev))
    b.forward(4, None)
    ref, _ = b.get_state()
    flat = w.X.copy()
    flat[:, :, 2] = 0.0
    with pytest.raises(C.MPMError) as ei:
        b.set_rest(torch.from_numpy(flat).to(dev))
    assert ei.value.code == C.MPM_BAD_STATE
    b.set_state(torch.from_numpy(w.x0).to(dev))
    b.forward(4, None)
    again, _ = b.get_state()
    assert torch.equal(ref, again)
    # a non-finite state is reported per env
    x = torch.from_numpy(w.x0).to(dev).clone()
    x[1, 3, 0] = float("nan")
    b.set_state(x)
    b.forward(2, None)
    assert b.sync(raise_on_error=False) == C.MPM_NONFINITE
    assert list(b.env_errors()) == [0, 1]
    assert b.sync(raise_on_error=False) == C.MPM_OK
    b.close()


def test_autograd_function_matches_oracle():
    from paper_2412_12089_amd.fem import rollout
    dev = torch.device("cuda:0")
    w = FS.two_cubes(seed=9, n_envs=2, substeps=8)
    b = make_batch(w)
    x0 = torch.from_numpy(w.x0).to(dev).requires_grad_(True)
    v0 = torch.from_numpy(w.v0).to(dev).requires_grad_(True)
    act = torch.from_numpy(w.act).to(dev).requires_grad_(True)
    prm = torch.from_numpy(w.params).requires_grad_(True)   # float64 on the host
    x, v = rollout(b, w.substeps, x0, v0, act, prm)
    wx = torch.linspace(-1, 1, x.numel(), device=dev).reshape(x.shape)
    (x * wx).sum().backward()
    for e in range(w.n_envs):
        og = FO.rollout_vjp(FO.Mesh(w.tets), w.X[e], w.params[e], w.x0[e], w.v0[e], w.act[:, e], w.substeps, w.dt,
                            wx[e].cpu().numpy(), np.zeros_like(w.x0[e]))
        assert relerr(x0.grad[e].cpu().numpy(), og[0].numpy()) < TOL_GRAD
        assert relerr(v0.grad[e].cpu().numpy(), og[1].numpy()) < TOL_GRAD
        assert relerr(act.grad[:, e].cpu().numpy(), og[2].numpy()) < TOL_GRAD
        assert relerr(prm.grad[e, :2].numpy(), og[3][:2].numpy()) < TOL_GRAD
    b.close()
