"""Parity of the HIP path (through the C interface) against the FP64 oracle.

Tolerances (normwise per environment, ||a - b|| / ||b||): positions and
velocities 1e-5 after the rollout, C and F 1e-4, gradients 1e-3, parameter
cotangents 1e-3 relative. Beside each normwise check: every particle within
ten times that bar (relative to the env's rms magnitude), and the displacement
x - x0 normwise within 1e-3. Binning keys and the sort permutation are
bit-exact.
"""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import (assert_grads, assert_params, assert_state, env_slices, gpu_rollout, make_env, oracle_rollout,
                      random_cotangents, relerr, to_np)
from oracle import mpm_oracle as O
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL_GRAD = 1e-3


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def check_state(g, o, tag, x0, S):
    assert_state(g, o, x0, tag, announce, S=S)


def check_grads(g, o, tag):
    assert_grads(g, o, tag, announce)


def check_params(gp, op, idx, tag, prm):
    assert_params(gp, op, idx, tag, prm, announce)


# ------------------------------------------------------------------ a2: binning
def test_keys_and_permutation_bit_exact():
    from paper_2412_12089_amd.batch import Batch
    rng = np.random.Generator(np.random.PCG64(7))
    envs = []
    for n, N in ((32, 3000), (48, 5000), (64, 700)):
        e = make_env(scenes.NEOHOOKEAN, N=N, n=n, seed=n)
        # positions exactly on cell boundaries (x n - 1/2 integral) and one ulp either side
        k = rng.integers(3, n - 4, size=(N // 3, 3))
        xb = ((k + 0.5) / n).astype(np.float32)
        which = rng.integers(0, 3, size=xb.shape)
        xb = np.where(which == 1, np.nextafter(xb, np.float32(0)), xb)
        xb = np.where(which == 2, np.nextafter(xb, np.float32(1)), xb)
        e.x[: len(xb)] = xb
        e.x[len(xb): len(xb) + 5] = e.x[len(xb) + 10]  # repeated keys: stability matters
        envs.append(e)
    announce("keys/permutation on 3 envs (32^3, 48^3, 64^3) with boundary positions")
    b = Batch(envs, max_substeps=1, ckpt_every=1)
    b.set_particles_from_specs()
    keys, perm, ids, cell_bits = b.sort_keys()
    b.sync()
    b.close()
    mask = (1 << cell_bits) - 1
    for i, (e, sl) in enumerate(zip(envs, env_slices(envs))):
        ok = O.cell_keys(e.x, e.n)
        assert np.array_equal(keys[sl] & mask, ok)
        assert np.all((keys[sl] >> cell_bits) == i)
        assert np.array_equal(perm[sl] - sl.start, O.sort_permutation(ok))
        assert np.array_equal(ids[sl], np.arange(0, sl.stop - sl.start))   # env-local caller index


# ------------------------------------------------------------------ config 1 (single env, neo-Hookean)
@pytest.mark.parametrize("mode", ["plain", "batched"])
def test_single_nh_forward_and_gradient(mode):
    wl = scenes.single_nh()
    spec = wl.envs[0]
    S = wl.substeps
    announce(f"single_nh {mode}: N={spec.n_particles} S={S}")
    cot = (wl.loss_weights[0], np.zeros((spec.n_particles, 3), np.float32),
           np.zeros((spec.n_particles, 3, 3), np.float32), np.zeros((spec.n_particles, 3, 3), np.float32))
    g = gpu_rollout(wl.envs, S, K=5, mode=mode, cots=[cot])
    o = oracle_rollout(spec, S, cot)
    assert g["status"] == 0
    check_state(g["state"], o["state"], f"single_nh {mode}", spec.x, S)
    ev = relerr(g["grads"][1], o["grads"][1])
    ex = relerr(g["grads"][0], o["grads"][0])
    announce(f"single_nh {mode}: dL/dv0 {ev:.2e} dL/dx0 {ex:.2e}")
    assert ev < TOL_GRAD and ex < TOL_GRAD
    check_params(g["dparams"][0], o["dparams"], [0, 2, 3], f"single_nh {mode}", spec.params())


# ------------------------------------------------------------------ every material, several segments
MATERIAL_CASES = [
    (scenes.NEOHOOKEAN, dict(F_dev=0.02), [0, 1]),
    (scenes.COROTATED, dict(F_dev=0.02, E=1e4, nu=0.25), [0, 1]),
    (scenes.VONMISES, dict(F_dev=(0.01, 0.0003), nu=0.2, sigma_y=5.0), [0, 1, 4]),
    (scenes.FLUID_TAIT, dict(), [5, 6]),
    (scenes.FLUID_PAPER, dict(E=2e3, nu=0.3), [0, 1]),
]


@pytest.mark.parametrize("mat,kw,pidx", MATERIAL_CASES, ids=[scenes.MATERIAL_NAMES[m[0]] for m in MATERIAL_CASES])
@pytest.mark.parametrize("mode", ["plain", "batched", "batched-fused"])
def test_material_forward_and_gradient(mat, kw, pidx, mode):
    spec = make_env(mat, N=2500, seed=10 + mat, **kw)
    S, K = 8, 3
    announce(f"{scenes.MATERIAL_NAMES[mat]} {mode}: N={spec.n_particles} S={S} K={K}")
    cots = random_cotangents([spec], seed=20 + mat)
    g = gpu_rollout([spec], S, K, mode=mode, cots=cots)
    o = oracle_rollout(spec, S, cots[0])
    assert g["status"] == 0
    check_state(g["state"], o["state"], scenes.MATERIAL_NAMES[mat], spec.x, S)
    check_grads(g["grads"], o["grads"], scenes.MATERIAL_NAMES[mat])
    check_params(g["dparams"][0], o["dparams"], pidx + [2, 3], scenes.MATERIAL_NAMES[mat], spec.params())


def test_von_mises_case_is_plastic():
    spec = make_env(scenes.VONMISES, N=2500, seed=10 + scenes.VONMISES, F_dev=(0.01, 0.0003), nu=0.2, sigma_y=5.0)
    env, prm, (x, v, C, F) = O.env_from_spec(spec)
    mu, _ = O.lame(prm[0], prm[1])
    Fp = O.project(O.VONMISES, F, mu, prm[4])
    moved = int(((Fp - F).flatten(1).norm(dim=1) > 1e-12).sum())
    assert 0 < moved < len(F)


# ------------------------------------------------------------------ contact with a moving box
def test_box_collider_forward_and_gradient():
    box = scenes.BoxCollider(center=(0.62, 0.46, 0.46), half=(0.04, 0.2, 0.2), velocity=(-0.5, 0.0, 0.0),
                             alpha=64.0, mu_b=0.5)
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=40, collider=box, v_scale=0.2)
    S, K = 10, 4
    announce(f"tait + moving box: N={spec.n_particles} S={S} K={K}")
    cots = random_cotangents([spec], seed=41)
    g = gpu_rollout([spec], S, K, cots=cots)
    o = oracle_rollout(spec, S, cots[0])
    check_state(g["state"], o["state"], "collider", spec.x, S)
    check_grads(g["grads"], o["grads"], "collider")
    check_params(g["dparams"][0], o["dparams"], [5, 2, 3], "collider", spec.params())


# ------------------------------------------------------------------ a box driven by per-substep velocities
BOXES = {   # the particles meet the box's face, or slide past one of its edges (normal turning with the center)
    "face": scenes.BoxCollider(center=(0.62, 0.46, 0.46), half=(0.04, 0.2, 0.2), velocity=(-0.5, 0.0, 0.0),
                               alpha=64.0, mu_b=0.5),
    "edge": scenes.BoxCollider(center=(0.61, 0.63, 0.46), half=(0.04, 0.07, 0.2), velocity=(-0.4, -0.3, 0.0),
                               alpha=64.0, mu_b=0.3),
}


def test_edge_box_has_sliding_edge_nodes():
    # the oracle's view of the edge case: some active nodes are outside two faces at once and slide
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=44, collider=BOXES["edge"], v_scale=0.2)
    env, prm, (x, v, C, F) = O.env_from_spec(spec)
    gm, gP, _ = O.p2g(env, prm, x, v, C, F)
    pos = gm > 0
    center, vb = O.collider_motion(env, 0.0)[:2]
    rel = O.node_positions(env.n) - center
    q = rel.abs() - torch.tensor(env.collider.half, dtype=torch.float64)
    d, nh = O.box_sdf(O.node_positions(env.n), center, torch.tensor(env.collider.half, dtype=torch.float64))
    vel = torch.where(pos[:, None], gP / torch.where(pos, gm, torch.ones_like(gm))[:, None], torch.zeros_like(gP))
    u = vel - vb
    un = (u * nh).sum(1)
    ut = (u - un[:, None] * nh).norm(dim=1)
    edge = pos & ((q > 0).sum(1) >= 2) & (un < 0) & (ut > -env.collider.mu_b * un) & (d < 4.0 / env.collider.alpha)
    assert int(edge.sum()) > 0


def set_pull_schedule(b):
    """The low particles-per-cell schedule: pull scatters, both fusions, the flagged-tile list."""
    from paper_2412_12089_amd import _capi as C
    for opt, val in ((C.OPT_P2G, 3), (C.OPT_G2P_ADJ, 3), (C.OPT_FUSE, 1), (C.OPT_FUSE_ADJ, 1), (C.OPT_GRID_LIST, 1)):
        b.set_option(opt, val)


@pytest.mark.parametrize("geom", ["face", "edge"])
@pytest.mark.parametrize("mode", ["plain", "batched", "batched-fused", "batched-pull"])
def test_collider_actions_forward_and_gradient(mode, geom):
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    box = BOXES[geom]
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=44, collider=box, v_scale=0.2)
    other = make_env(scenes.NEOHOOKEAN, N=1200, seed=45)   # no prescribed motion, same batch
    S, K = 10, 4
    rng = np.random.default_rng(46)
    vel = (np.array(box.velocity) + 0.3 * rng.standard_normal((S, 3))).astype(np.float32)
    announce(f"tait + box ({geom}) driven by {S} actions, {mode}")
    envs = [spec, other]
    cots = random_cotangents(envs, seed=47)
    b = Batch(envs, max_substeps=S, ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode == "batched-fused":   # the fused G2P + P2G and adjoint-pair schedules
            b.set_option(C.OPT_FUSE, 1)
            b.set_option(C.OPT_FUSE_ADJ, 1)
        if mode == "batched-pull":    # the pull scatters, both fusions, grid passes over the flagged-tile list
            set_pull_schedule(b)
        b.set_particles_from_specs()
        b.set_collider_motion(0, vel)
        b.forward(S, record=True)
        st = tuple(to_np(t) for t in b.get_particles(env=0))
        cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
        dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
        N0 = spec.n_particles
        gr = tuple(to_np(t)[:N0] for t in (dx, dv, dC, dF))
        dvel, dc0 = b.collider_grad(0, S)
        assert b.sync(raise_on_error=False) == 0
        with pytest.raises(Exception):
            b.collider_grad(1, S)          # env 1 has no prescribed motion
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    velt = torch.from_numpy(vel).double()
    (x, v, C, F), _ = O.rollout(env, prm, st0, S, vel=velt)
    c = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).double() for a in cots[0])
    g, gp, gvel, gc0 = O.rollout_vjp(env, prm, st0, S, c, vel=velt)
    check_state(st, tuple(t.numpy() for t in (x, v, C, F)), "actions", spec.x, S)
    check_grads(gr, tuple(t.numpy() for t in g), "actions")
    ev, ec = relerr(dvel, gvel.numpy()), relerr(dc0, gc0.numpy())
    announce(f"actions: dL/dvel rel {ev:.2e}, dL/dc0 rel {ec:.2e}, |dL/dvel| {np.abs(gvel.numpy()).max():.3e}")
    assert np.abs(gvel.numpy()).max() > 0
    assert ev < 1e-3 and ec < 1e-3


SPIN_BOX = scenes.BoxCollider(center=(0.6, 0.46, 0.46), half=(0.04, 0.12, 0.2), velocity=(-0.4, 0.0, 0.0),
                              alpha=64.0, mu_b=0.3, axis=(0.0, 0.6, 0.8), angle=0.4, omega=6.0)


@pytest.mark.parametrize("mode", ["plain", "batched", "batched-fused", "batched-pull"])
def test_spinning_box_forward_and_gradient(mode):
    # a box turned about a tilted axis and spinning at a constant rate, against the oracle
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=160, collider=SPIN_BOX, v_scale=0.2)
    S, K = 10, 4
    announce(f"tait + spinning box (constant rate), {mode}")
    cots = random_cotangents([spec], seed=161)
    g = gpu_rollout([spec], S, K, mode=mode, cots=cots)
    o = oracle_rollout(spec, S, cots[0])
    assert g["status"] == 0
    check_state(g["state"], o["state"], "spinning box", spec.x, S)
    check_grads(g["grads"], o["grads"], "spinning box")
    check_params(g["dparams"][0], o["dparams"], [5, 2, 3], "spinning box", spec.params())


@pytest.mark.parametrize("mode", ["plain", "batched", "batched-fused", "batched-pull"])
def test_spin_actions_forward_and_gradient(mode):
    # per-substep velocities and angular speeds drive the turned box; gradients w.r.t. both, the
    # starting center and the starting angle against the oracle
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=162, collider=SPIN_BOX, v_scale=0.2)
    other = make_env(scenes.NEOHOOKEAN, N=1000, seed=163)
    S, K = 10, 4
    rng = np.random.default_rng(164)
    vel = (np.array(SPIN_BOX.velocity) + 0.3 * rng.standard_normal((S, 3))).astype(np.float32)
    om = (SPIN_BOX.omega + 4.0 * rng.standard_normal(S)).astype(np.float32)
    announce(f"spinning box driven by {S} velocity and angular-speed actions, {mode}")
    envs = [spec, other]
    cots = random_cotangents(envs, seed=165)
    b = Batch(envs, max_substeps=S, ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode == "batched-fused":
            b.set_option(C.OPT_FUSE, 1)
            b.set_option(C.OPT_FUSE_ADJ, 1)
        if mode == "batched-pull":
            set_pull_schedule(b)
        b.set_particles_from_specs()
        b.set_collider_motion(0, vel, om)
        b.forward(S, record=True)
        st = tuple(to_np(t) for t in b.get_particles(env=0))
        cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
        dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
        N0 = spec.n_particles
        gr = tuple(to_np(t)[:N0] for t in (dx, dv, dC, dF))
        dvel, dc0, dom, dang = b.collider_grad(0, S, spin=True)
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    velt, omt = torch.from_numpy(vel).double(), torch.from_numpy(om).double()
    (x, v, Cm, F), _ = O.rollout(env, prm, st0, S, vel=velt, omega=omt)
    c = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).double() for a in cots[0])
    g, gp, gvel, gc0, gom, gang = O.rollout_vjp(env, prm, st0, S, c, vel=velt, omega=omt)
    check_state(st, tuple(t.numpy() for t in (x, v, Cm, F)), "spin actions", spec.x, S)
    check_grads(gr, tuple(t.numpy() for t in g), "spin actions")
    ev, ec, eo = relerr(dvel, gvel.numpy()), relerr(dc0, gc0.numpy()), relerr(dom, gom.numpy())
    ea = abs(dang - float(gang)) / abs(float(gang))
    announce(f"spin actions: dL/dvel {ev:.2e}, dL/dc0 {ec:.2e}, dL/domega {eo:.2e}, dL/dangle0 {ea:.2e}, "
             f"|dL/domega| {np.abs(gom.numpy()).max():.3e}")
    assert np.abs(gom.numpy()).max() > 0 and abs(float(gang)) > 0
    assert ev < 1e-3 and ec < 1e-3 and eo < 1e-3 and ea < 1e-3


SPIN_BALL = scenes.sphere_collider(center=(0.62, 0.5, 0.48), radius=0.1, velocity=(-0.4, 0.0, 0.0), alpha=64.0,
                                   mu_b=0.3, axis=(0.0, 0.6, 0.8), angle=0.4, omega=6.0)
# a finger: a capsule along its own x axis, turned about a tilted axis and spinning
SPIN_CAPSULE = scenes.capsule_collider(center=(0.6, 0.47, 0.47), half_length=0.1, radius=0.04,
                                       velocity=(-0.4, 0.0, 0.0), alpha=64.0, mu_b=0.3, axis=(0.6, 0.0, 0.8),
                                       angle=1.2, omega=5.0)
ROUNDED = {"ball": SPIN_BALL, "capsule": SPIN_CAPSULE}


@pytest.mark.parametrize("geom", ["ball", "capsule"])
@pytest.mark.parametrize("mode", ["plain", "batched", "batched-fused", "batched-pull"])
def test_rounded_collider_actions_forward_and_gradient(mode, geom):
    # a spinning ball or capsule driven by per-substep velocities and angular speeds (their normals turn with
    # the nodes' positions relative to the center or the segment); gradients w.r.t. both actions, the
    # starting center and the starting angle against the oracle (none for the ball's angle, which moves
    # nothing)
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    col = ROUNDED[geom]
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=170, collider=col, v_scale=0.2)
    other = make_env(scenes.NEOHOOKEAN, N=1000, seed=171, collider=BOXES["face"])   # a box in the same batch
    S, K = 10, 4
    rng = np.random.default_rng(172)
    vel = (np.array(col.velocity) + 0.3 * rng.standard_normal((S, 3))).astype(np.float32)
    om = (col.omega + 4.0 * rng.standard_normal(S)).astype(np.float32)
    announce(f"spinning {geom} driven by {S} velocity and angular-speed actions, {mode}")
    envs = [spec, other]
    cots = random_cotangents(envs, seed=173)
    b = Batch(envs, max_substeps=S, ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode == "batched-fused":
            b.set_option(C.OPT_FUSE, 1)
            b.set_option(C.OPT_FUSE_ADJ, 1)
        if mode == "batched-pull":
            set_pull_schedule(b)
        b.set_particles_from_specs()
        b.set_collider_motion(0, vel, om)
        b.forward(S, record=True)
        st = tuple(to_np(t) for t in b.get_particles(env=0))
        cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
        dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
        N0 = spec.n_particles
        gr = tuple(to_np(t)[:N0] for t in (dx, dv, dC, dF))
        dvel, dc0, dom, dang = b.collider_grad(0, S, spin=True)
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    assert env.collider.shape == ("sphere" if geom == "ball" else "box") and (geom == "ball") == (env.collider.rounding == 0)
    velt, omt = torch.from_numpy(vel).double(), torch.from_numpy(om).double()
    (x, v, Cm, F), _ = O.rollout(env, prm, st0, S, vel=velt, omega=omt)
    c = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).double() for a in cots[0])
    g, gp, gvel, gc0, gom, gang = O.rollout_vjp(env, prm, st0, S, c, vel=velt, omega=omt)
    check_state(st, tuple(t.numpy() for t in (x, v, Cm, F)), f"{geom} actions", spec.x, S)
    check_grads(gr, tuple(t.numpy() for t in g), f"{geom} actions")
    ev, ec, eo = relerr(dvel, gvel.numpy()), relerr(dc0, gc0.numpy()), relerr(dom, gom.numpy())
    announce(f"{geom} actions: dL/dvel {ev:.2e}, dL/dc0 {ec:.2e}, dL/domega {eo:.2e}, dL/dangle0 {dang:.2e} "
             f"(oracle {float(gang):.2e}), |dL/domega| {np.abs(gom.numpy()).max():.3e}")
    assert np.abs(gom.numpy()).max() > 0
    assert ev < 1e-3 and ec < 1e-3 and eo < 1e-3
    if geom == "ball":
        assert float(gang) == 0.0 and abs(dang) < 1e-3 * float(np.linalg.norm(gc0.numpy()))
    else:
        assert abs(float(gang)) > 0 and abs(dang - float(gang)) < 1e-3 * abs(float(gang))


def test_sphere_collider_has_sliding_curved_contacts():
    # the oracle's view: active nodes inside the ball's contact band that slide, where the normal differs
    # from node to node (so the normal's dependence on the center is exercised)
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=170, collider=SPIN_BALL, v_scale=0.2)
    env, prm, (x, v, C, F) = O.env_from_spec(spec)
    gm, gP, _ = O.p2g(env, prm, x, v, C, F)
    pos = gm > 0
    center, vb = O.collider_motion(env, 0.0)[:2]
    d, nh = O.sphere_sdf(O.node_positions(env.n), center, env.collider.half[0])
    vel = torch.where(pos[:, None], gP / torch.where(pos, gm, torch.ones_like(gm))[:, None], torch.zeros_like(gP))
    u = vel - vb
    un = (u * nh).sum(1)
    ut = (u - un[:, None] * nh).norm(dim=1)
    slide = pos & (un < 0) & (ut > -env.collider.mu_b * un) & (d < 4.0 / env.collider.alpha)
    assert int(slide.sum()) > 10
    assert float(nh[slide].std(0).norm()) > 0.1


def test_rollout_function_with_spins_matches_oracle():
    # the autograd Function carries the angular-speed actions' gradient
    from paper_2412_12089_amd.batch import Batch, rollout
    spec = make_env(scenes.FLUID_TAIT, N=2000, seed=166, collider=SPIN_BOX, v_scale=0.2)
    S, K = 6, 3
    dev = torch.device("cuda:0")
    st = [torch.from_numpy(getattr(spec, k)).to(dev) for k in ("x", "v", "C", "F")]
    params = torch.tensor(spec.params()[None], dtype=torch.float64)
    rng = np.random.default_rng(167)
    vel = torch.from_numpy((np.array(SPIN_BOX.velocity) + 0.3 * rng.standard_normal((1, S, 3))).astype(np.float32))
    spins = torch.from_numpy((SPIN_BOX.omega + 4.0 * rng.standard_normal((1, S))).astype(np.float32)).requires_grad_(True)
    w = torch.from_numpy(rng.standard_normal((spec.n_particles, 3)).astype(np.float32)).to(dev)
    b = Batch([spec], max_substeps=S, ckpt_every=K)
    try:
        xs, _, _, _ = rollout(b, S, *st, params, vel, None, spins)
        (xs * w).sum().backward()
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    cot = (torch.from_numpy(w.cpu().numpy()).double(), None, None, None)
    _, _, _, _, gom, _ = O.rollout_vjp(env, prm, st0, S, cot, vel=vel[0].double(), omega=spins[0].detach().double())
    e = relerr(spins.grad[0].numpy(), gom.numpy())
    announce(f"rollout Function: dL/dspins {e:.2e}")
    assert e < 1e-3


def test_collider_actions_bounds():
    from paper_2412_12089_amd.batch import Batch
    from paper_2412_12089_amd._capi import MPMError
    box = scenes.BoxCollider(center=(0.62, 0.46, 0.46), half=(0.04, 0.2, 0.2), velocity=(-0.5, 0.0, 0.0),
                             alpha=64.0, mu_b=0.5)
    spec = make_env(scenes.FLUID_TAIT, N=500, seed=48, collider=box)
    b = Batch([spec], max_substeps=6, ckpt_every=3)
    try:
        b.set_particles_from_specs()
        b.set_collider_motion(0, np.zeros((4, 3), np.float32))
        with pytest.raises(MPMError):
            b.forward(6)                    # the motion covers 4 substeps only
        b.forward(4)
        with pytest.raises(MPMError):
            b.set_collider_motion(0, np.full((2, 3), np.nan, np.float32))
        b.set_collider_motion(0, None)      # back to the constant velocity
        b.forward(2)
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()


def test_collider_clocks_are_per_env():
    # two envs with moving boxes; setting one env's particles again restarts only that env's clock
    # (its box returns to its t = 0 position), the other env's box keeps moving; the backward of the
    # next recorded forward places each box at its own time
    from paper_2412_12089_amd.batch import Batch
    box = BOXES["face"]
    a = make_env(scenes.FLUID_TAIT, N=2500, seed=150, collider=box, v_scale=0.2)
    c = make_env(scenes.FLUID_TAIT, N=1800, seed=151, collider=box, v_scale=0.2)
    S1, S2, K = 4, 6, 4
    cots = random_cotangents([a, c], seed=152)
    announce(f"per-env collider clocks: {S1} substeps, env 1 reset, then {S2} recorded substeps")
    b = Batch([a, c], max_substeps=S2, ckpt_every=K)
    try:
        b.set_particles_from_specs()
        b.forward(S1)
        b.set_particles(*(torch.from_numpy(getattr(c, k)) for k in ("x", "v", "C", "F")), env=1)
        b.forward(S2, record=True)
        st = [to_np(t) for t in b.get_particles()]
        cat = lambda k: torch.from_numpy(np.concatenate([q[k] for q in cots], axis=0))
        dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
        gr = [to_np(t) for t in (dx, dv, dC, dF)]
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()
    sl = env_slices([a, c])
    # env 0: S1 substeps, then S2 more with the box at t = S1 dt (oracle continues from its own state)
    env, prm, st0 = O.env_from_spec(a)
    mid, _ = O.rollout(env, prm, st0, S1)
    (x, v, C, F), _ = O.rollout(env, prm, mid, S2, t0=S1 * a.dt)
    cot0 = tuple(torch.from_numpy(np.asarray(q, dtype=np.float32)).double() for q in cots[0])
    g0, _ = O.rollout_vjp(env, prm, mid, S2, cot0, t0=S1 * a.dt)
    check_state([s[sl[0]] for s in st], tuple(t.numpy() for t in (x, v, C, F)), "clock env 0 (t0 = 4 dt)",
                a.x, S1 + S2)
    check_grads([g[sl[0]] for g in gr], tuple(t.numpy() for t in g0), "clock env 0 (t0 = 4 dt)")
    # env 1: S2 substeps from its initial state with the box at t = 0
    o1 = oracle_rollout(c, S2, cots[1])
    check_state([s[sl[1]] for s in st], o1["state"], "clock env 1 (restarted)", c.x, S2)
    check_grads([g[sl[1]] for g in gr], o1["grads"], "clock env 1 (restarted)")


# ------------------------------------------------------------------ batching and checkpoint invariances
def test_env_in_batch_equals_env_alone():
    a = make_env(scenes.NEOHOOKEAN, N=1500, n=32, seed=50)
    b = make_env(scenes.VONMISES, N=2600, n=48, seed=51, sigma_y=5.0, nu=0.2)
    c = make_env(scenes.FLUID_TAIT, N=900, n=32, seed=52)
    envs = [a, b, c]
    S, K = 6, 4
    announce("batch of 3 uneven envs vs each alone")
    cots = random_cotangents(envs, seed=53)
    together = gpu_rollout(envs, S, K, cots=cots)
    for i, (e, sl) in enumerate(zip(envs, env_slices(envs))):
        alone = gpu_rollout([e], S, K, cots=[cots[i]])
        for j in range(4):
            assert relerr(together["state"][j][sl], alone["state"][j]) < 1e-6
            assert relerr(together["grads"][j][sl], alone["grads"][j]) < 1e-4   # FP32 atomic order
        # E, nu, rho, sigma_y, K, gamma (the Vp cotangent is exactly 0 on both)
        sel = [0, 1, 2, 4, 5, 6]
        assert together["dparams"][i][3] == 0.0 and alone["dparams"][0][3] == 0.0
        assert np.allclose(together["dparams"][i][sel], alone["dparams"][0][sel], rtol=1e-4, atol=0)


def test_checkpoint_interval_does_not_change_gradients():
    spec = make_env(scenes.COROTATED, N=2000, seed=60, F_dev=0.02)
    S = 9
    cots = random_cotangents([spec], seed=61)
    announce("checkpoint intervals 1, 4, 9")
    runs = [gpu_rollout([spec], S, K, cots=cots) for K in (1, 4, 9)]
    for r in runs[1:]:
        for j in range(4):
            assert relerr(r["state"][j], runs[0]["state"][j]) < 1e-6
            assert relerr(r["grads"][j], runs[0]["grads"][j]) < 1e-5


def test_identical_envs_get_identical_parameter_gradients():
    spec = make_env(scenes.COROTATED, N=1500, seed=70, F_dev=0.02)
    envs = [spec.copy() for _ in range(4)]
    cots = random_cotangents([spec], seed=71) * 4
    r = gpu_rollout(envs, 5, 5, cots=cots)
    dE = r["dparams"][:, 0]
    assert np.allclose(dE, dE[0], rtol=1e-4)


# ------------------------------------------------------------------ status codes from the device
def test_out_of_domain_is_reported_and_clamped():
    spec = make_env(scenes.NEOHOOKEAN, N=500, seed=80)
    spec.x[0] = np.float32([0.01, 0.5, 0.5])   # below the 0.5/n band
    announce("out-of-domain particle")
    r = gpu_rollout([spec], 2, 2)
    assert r["status"] == 5
    assert r["errors"][0] & 2


def test_backward_needs_a_recorded_forward():
    from paper_2412_12089_amd.batch import Batch
    from paper_2412_12089_amd._capi import MPMError
    spec = make_env(scenes.NEOHOOKEAN, N=300, seed=81)
    b = Batch([spec], max_substeps=4, ckpt_every=2)
    b.set_particles_from_specs()
    b.forward(2, record=False)
    with pytest.raises(MPMError) as ei:
        b.backward(gx=torch.zeros(300, 3))
    assert ei.value.code == 6
    with pytest.raises(MPMError) as ei:
        b.forward(5)
    assert ei.value.code == 6
    b.sync()
    b.close()


# ------------------------------------------------------------------ per-env substep counts and slot reuse
@pytest.mark.parametrize("counts", [[7, 3], [7, 4]], ids=["stop-at-segment-end", "stop-inside-segment"])
@pytest.mark.parametrize("fused", [0, 1, 2], ids=["unfused", "fused", "pull-fused"])
def test_per_env_substep_counts_match_separate_runs(counts, fused):
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    a = make_env(scenes.NEOHOOKEAN, N=1200, n=32, seed=90)
    b_ = make_env(scenes.COROTATED, N=1800, n=32, seed=91, F_dev=0.02)
    envs = [a, b_]
    cots = random_cotangents(envs, seed=92)
    announce(f"forward_envs with counts {counts} (fused kernels {fused}) vs separate runs")
    bt = Batch(envs, max_substeps=8, ckpt_every=3)
    bt.set_option(C.OPT_FUSE, 1 if fused else 0)
    bt.set_option(C.OPT_FUSE_ADJ, 1 if fused else 0)
    if fused == 2:   # the pull scatters, both fusions (G2P + pull P2G, P2G adjoint + pull G2P adjoint)
        bt.set_option(C.OPT_P2G, 3)
        bt.set_option(C.OPT_G2P_ADJ, 3)
    bt.set_particles_from_specs()
    bt.forward_envs(counts, record=True)
    st = [t.cpu().double().numpy() for t in bt.get_particles()]
    cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
    dx, dv, dC, dF, dp = bt.backward(cat(0), cat(1), cat(2), cat(3))
    gr = [t.cpu().double().numpy() for t in (dx, dv, dC, dF)]
    assert bt.sync(raise_on_error=False) == 0
    bt.close()
    for i, (e, sl) in enumerate(zip(envs, env_slices(envs))):
        alone = gpu_rollout([e], counts[i], 3, cots=[cots[i]])
        for j in range(4):
            assert relerr(st[j][sl], alone["state"][j]) < 1e-6, (i, j)
            assert relerr(gr[j][sl], alone["grads"][j]) < 1e-4, (i, j)


def test_slot_reconfiguration_matches_oracle():
    from paper_2412_12089_amd.batch import Batch
    cap = [make_env(scenes.NEOHOOKEAN, N=4000, n=48, seed=93), make_env(scenes.NEOHOOKEAN, N=4000, n=48, seed=94)]
    bt = Batch(cap, max_substeps=6, ckpt_every=3)
    rounds = [
        [make_env(scenes.NEOHOOKEAN, N=2500, n=32, seed=95), make_env(scenes.VONMISES, N=3000, n=48, seed=96,
                                                                      F_dev=(0.01, 0.0003), nu=0.2, sigma_y=5.0)],
        [make_env(scenes.FLUID_TAIT, N=1000, n=48, seed=97, lo=0.4, side=0.15), None],
    ]
    S = 5
    for r, specs in enumerate(rounds):
        for i, sp in enumerate(specs):
            if sp is not None:
                bt.configure_env(i, sp)
                bt.set_particles(*(torch.from_numpy(getattr(sp, k)) for k in ("x", "v", "C", "F")), env=i)
        live = [sp if sp is not None else rounds[r - 1][i] for i, sp in enumerate(specs)]
        announce(f"slot round {r}: " + ", ".join(f"{scenes.MATERIAL_NAMES[s.material]} n={s.n} N={s.n_particles}" for s in live))
        bt.forward(S, record=True)
        st = [t.cpu().double().numpy() for t in bt.get_particles()]
        cots = random_cotangents(live, seed=98 + r)
        cat = lambda k: torch.from_numpy(np.concatenate([c[k] for c in cots], axis=0))
        dx, dv, dC, dF, dp = bt.backward(cat(0), cat(1), cat(2), cat(3))
        gr = [t.cpu().double().numpy() for t in (dx, dv, dC, dF)]
        assert bt.sync(raise_on_error=False) == 0
        for i, (sp, sl) in enumerate(zip(live, env_slices(live))):
            if r == 1 and i == 1:
                continue   # slot 1 kept running from its round-0 end state
            o = oracle_rollout(sp, S, cots[i])
            check_state([s[sl] for s in st], o["state"], f"slot {i} round {r}", sp.x, S)
            check_grads([g[sl] for g in gr], o["grads"], f"slot {i} round {r}")
    bt.close()


# ------------------------------------------------------------------ kernel variants and the autotuner
VARIANTS = [  # (P2G, G2P, G2P adjoint, P2G adjoint, grid cap, small LDS box, per-material launches,
              #  fused G2P+P2G, fused P2G adjoint + G2P adjoint[, XCD-ordered items[, flagged-tile list]])
    (0, 0, 0, 0, 0, 0, 1, 0, 0), (1, 1, 1, 1, 0, 0, 1, 0, 0), (2, 1, 2, 1, 0, 0, 1, 0, 0), (2, 1, 2, 1, 7, 0, 1, 0, 0),
    (1, 0, 2, 0, 3, 0, 1, 0, 0), (1, 1, 1, 1, 0, 1, 1, 0, 0), (2, 1, 2, 1, 0, 1, 1, 0, 0), (2, 1, 2, 1, 5, 1, 1, 0, 0),
    (1, 1, 1, 1, 0, 0, 0, 0, 0), (2, 1, 2, 1, 6, 1, 0, 0, 0), (2, 0, 2, 1, 0, 1, 1, 1, 0), (2, 1, 2, 1, 0, 0, 0, 1, 0),
    (2, 0, 2, 1, 0, 1, 1, 1, 1), (2, 1, 2, 1, 0, 0, 0, 1, 1), (0, 0, 0, 0, 0, 0, 1, 0, 1), (1, 1, 1, 1, 0, 1, 0, 0, 1),
    (2, 0, 2, 1, 0, 1, 1, 1, 1, 1), (2, 1, 2, 1, 0, 0, 0, 1, 1, 1), (1, 1, 1, 1, 3, 1, 1, 0, 0, 1),
    # owner-computes (pull) scatters through LDS: both box budgets, persistent grid, generic launch, XCD order
    (3, 1, 3, 1, 0, 0, 1, 0, 0), (3, 1, 3, 1, 0, 1, 1, 0, 0), (3, 0, 3, 0, 5, 0, 0, 0, 0), (3, 1, 3, 1, 0, 1, 0, 0, 0, 1),
    (3, 1, 3, 1, 0, 0, 1, 1, 1),
    # the pull P2G fused with the G2P, the P2G adjoint fused with the pull G2P adjoint: both box
    # budgets, generic launch, XCD order
    (3, 0, 3, 1, 0, 1, 1, 1, 0), (3, 1, 3, 1, 0, 0, 0, 1, 0), (3, 1, 3, 1, 0, 0, 1, 1, 0, 1),
    (3, 0, 3, 1, 0, 1, 1, 0, 1), (3, 1, 3, 1, 0, 0, 0, 1, 1), (3, 1, 3, 1, 0, 1, 0, 1, 1, 1),
    # the grid passes over the compact list of flagged tiles
    (3, 1, 3, 1, 0, 0, 1, 1, 1, 0, 1), (2, 1, 2, 1, 0, 0, 1, 1, 1, 0, 1), (0, 0, 0, 0, 0, 0, 1, 0, 0, 0, 1),
    (3, 1, 3, 1, 0, 0, 1, 1, 1, 0, 2), (2, 0, 2, 1, 0, 1, 1, 1, 1, 1, 2),
]


@pytest.mark.parametrize("var", VARIANTS, ids=["-".join(map(str, v)) for v in VARIANTS])
def test_every_kernel_variant_matches_oracle(var):
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    # ~6 and ~1.4 particles per cell, and a sparse env spread over the whole interior (~0.1 per cell,
    # whose blocks cross more tile rows than the LDS boxes hold: the global-atomic fallback)
    envs = [make_env(scenes.VONMISES, N=2200, seed=110, F_dev=(0.01, 0.0003), nu=0.2, sigma_y=5.0),
            make_env(scenes.COROTATED, N=1700, n=48, seed=111, F_dev=0.02),
            make_env(scenes.FLUID_TAIT, N=1500, n=32, seed=113, lo=0.12, side=0.76, v_scale=0.3)]
    S, K = 6, 4
    cots = random_cotangents(envs, seed=112)
    announce(f"variant {var}")
    b = Batch(envs, max_substeps=S, ckpt_every=K)
    for opt, val in zip((C.OPT_P2G, C.OPT_G2P, C.OPT_G2P_ADJ, C.OPT_P2G_ADJ, C.OPT_GRID_CAP, C.OPT_BOX, C.OPT_SPECIALIZE,
                         C.OPT_FUSE, C.OPT_FUSE_ADJ, C.OPT_XCD, C.OPT_GRID_LIST), var):
        b.set_option(opt, val)
    b.set_particles_from_specs()
    b.forward(S, record=True)
    st = [t.cpu().double().numpy() for t in b.get_particles()]
    cat = lambda k: torch.from_numpy(np.concatenate([c[k] for c in cots], axis=0))
    dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
    gr = [t.cpu().double().numpy() for t in (dx, dv, dC, dF)]
    assert b.sync(raise_on_error=False) == 0
    b.close()
    for i, (e, sl) in enumerate(zip(envs, env_slices(envs))):
        o = oracle_rollout(e, S, cots[i])
        check_state([a[sl] for a in st], o["state"], f"variant {var} env {i}", e.x, S)
        check_grads([g[sl] for g in gr], o["grads"], f"variant {var} env {i}")


def test_autotune_restores_state_and_keeps_parity():
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    envs = [make_env(scenes.COROTATED, N=3000, n=48, seed=120 + i, F_dev=0.02) for i in range(3)]
    b = Batch(envs, max_substeps=8, ckpt_every=4)
    b.set_particles_from_specs()
    before = [t.cpu().numpy() for t in b.get_particles()]
    announce("autotune on 3 corotated envs")
    b.autotune(3000)
    after = [t.cpu().numpy() for t in b.get_particles()]
    for a, c in zip(before, after):
        assert np.array_equal(a, c)
    opts = {k: b.get_option(getattr(C, k)) for k in ("OPT_P2G", "OPT_G2P", "OPT_G2P_ADJ", "OPT_P2G_ADJ", "OPT_GRID_CAP", "OPT_BOX", "OPT_SPECIALIZE")}
    announce(f"autotune chose {opts}")
    assert opts["OPT_P2G"] in (0, 1, 2, 3) and opts["OPT_GRID_CAP"] >= 0
    cots = random_cotangents(envs, seed=121)
    b.forward(8, record=True)
    st = [t.cpu().double().numpy() for t in b.get_particles()]
    cat = lambda k: torch.from_numpy(np.concatenate([c[k] for c in cots], axis=0))
    dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
    gr = [t.cpu().double().numpy() for t in (dx, dv, dC, dF)]
    assert b.sync(raise_on_error=False) == 0
    b.close()
    sl = env_slices(envs)[1]
    o = oracle_rollout(envs[1], 8, cots[1])
    check_state([a[sl] for a in st], o["state"], "after autotune", envs[1].x, 8)
    check_grads([g[sl] for g in gr], o["grads"], "after autotune")


# ------------------------------------------------------------------ failure forcing from the host
def test_nonfinite_input_is_reported():
    spec = make_env(scenes.NEOHOOKEAN, N=400, seed=130)
    spec.v[7] = np.float32([np.nan, 0.0, 0.0])
    announce("NaN velocity in the initial state")
    r = gpu_rollout([spec], 2, 2)
    assert r["status"] == 4
    assert r["errors"][0] & 1


def test_invalid_material_parameters_are_rejected():
    from paper_2412_12089_amd.batch import Batch
    from paper_2412_12089_amd._capi import MPMError
    spec = make_env(scenes.NEOHOOKEAN, N=100, seed=131)
    b = Batch([spec], max_substeps=2, ckpt_every=2)
    for bad in ([5e3, 0.5, 1e3, 1e-6, 0, 0, 0, 0], [-1.0, 0.3, 1e3, 1e-6, 0, 0, 0, 0],
                [5e3, -1.0, 1e3, 1e-6, 0, 0, 0, 0], [5e3, 0.3, -1.0, 1e-6, 0, 0, 0, 0]):
        with pytest.raises(MPMError) as ei:
            b.set_material(0, scenes.NEOHOOKEAN, bad)
        assert ei.value.code == 1
    with pytest.raises(MPMError):
        b.set_material(0, scenes.FLUID_TAIT, [0, 0.3, 1e3, 1e-6, 0, 1e4, 0.0, 0])   # gamma <= 0
    with pytest.raises(MPMError):
        b.set_material(0, 9, spec.params())
    with pytest.raises(MPMError):
        b.set_particles(torch.zeros(5, 3), torch.zeros(5, 3), torch.zeros(5, 3, 3), torch.zeros(5, 3, 3))
    b.close()


def test_checkpoint_memory_follows_segments_plus_tape():
    from paper_2412_12089_amd.batch import Batch
    spec = make_env(scenes.COROTATED, N=20000, seed=132)
    S = 36
    mem = {}
    for K in (1, 6, 36):
        b = Batch([spec], max_substeps=S, ckpt_every=K)
        mem[K] = b.memory_bytes()
        b.close()
    announce(f"memory bytes by K: {mem}")
    # state buffers ~ S/K checkpoints + K tape states (+ K tape grids): K = 6 is the minimum of S/K + K
    assert mem[6] < mem[1] and mem[6] < mem[36]


# ------------------------------------------------------------------ run-to-run spread (atomic reordering)
def test_run_to_run_spread_is_rounding_level():
    # float atomics add in a timing-dependent order, so two identical runs may differ in the last bits;
    # the spread is reported and must stay far below the parity bar; keys and permutations stay bit-exact
    envs = [make_env(scenes.COROTATED, N=4000, n=48, seed=80, F_dev=0.02, E=1e4, nu=0.25),
            make_env(scenes.FLUID_TAIT, N=3000, seed=81)]
    S, K = 12, 4
    cots = random_cotangents(envs, seed=82)
    a = gpu_rollout(envs, S, K, cots=cots)
    b = gpu_rollout(envs, S, K, cots=cots)
    st = max(relerr(x, y) for x, y in zip(a["state"], b["state"]))
    gr = max(relerr(x, y) for x, y in zip(a["grads"], b["grads"]))
    announce(f"run-to-run spread: state {st:.2e}, gradients {gr:.2e} "
             f"({'bit-identical' if st == 0 and gr == 0 else 'atomic reordering'})")
    assert st < 1e-6 and gr < 1e-5


# a gripper: a left jaw (a box), a right finger (a capsule, driven by actions) and a ball pressing from above
GRIP = (scenes.BoxCollider(center=(0.31, 0.46, 0.46), half=(0.04, 0.12, 0.12), velocity=(0.4, 0.0, 0.0),
                           alpha=64.0, mu_b=0.5),
        SPIN_CAPSULE,
        scenes.sphere_collider(center=(0.46, 0.46, 0.64), radius=0.06, velocity=(0.0, 0.0, -0.3), alpha=64.0,
                               mu_b=0.2, omega=-3.0))


@pytest.mark.parametrize("mode", ["plain", "batched", "batched-pull"])
def test_several_colliders_with_actions_forward_and_gradient(mode):
    # three colliders in one env, applied in turn by the grid update; the second one is driven by
    # per-substep velocities and angular speeds: states, state cotangents and the cotangents of that
    # collider's actions, start center and angle against the oracle; an env with one collider beside it
    import dataclasses
    from paper_2412_12089_amd.batch import Batch
    spec = make_env(scenes.FLUID_TAIT, N=3000, seed=180, collider=GRIP[0], v_scale=0.2)
    spec = dataclasses.replace(spec, more_colliders=GRIP[1:])
    other = make_env(scenes.NEOHOOKEAN, N=1000, seed=181, collider=BOXES["face"])
    S, K = 10, 4
    rng = np.random.default_rng(182)
    col = GRIP[1]
    vel = (np.array(col.velocity) + 0.3 * rng.standard_normal((S, 3))).astype(np.float32)
    om = (col.omega + 4.0 * rng.standard_normal(S)).astype(np.float32)
    announce(f"three colliders, the second driven by {S} actions, {mode}")
    envs = [spec, other]
    cots = random_cotangents(envs, seed=183)
    b = Batch(envs, max_substeps=S, ckpt_every=K, mode=mode.split("-")[0])
    try:
        if mode == "batched-pull":
            set_pull_schedule(b)
        b.set_particles_from_specs()
        b.set_collider_motion(0, vel, om, index=1)
        b.forward(S, record=True)
        st = tuple(to_np(t) for t in b.get_particles(env=0))
        cat = lambda i: torch.from_numpy(np.concatenate([c[i] for c in cots], axis=0))
        dx, dv, dC, dF, dp = b.backward(cat(0), cat(1), cat(2), cat(3))
        N0 = spec.n_particles
        gr = tuple(to_np(t)[:N0] for t in (dx, dv, dC, dF))
        dvel, dc0, dom, dang = b.collider_grad(0, S, spin=True, index=1)
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    assert len(env.colliders) == 3
    velt, omt = torch.from_numpy(vel).double(), torch.from_numpy(om).double()
    (x, v, Cm, F), _ = O.rollout(env, prm, st0, S, vel=velt, omega=omt, col=1)
    c = tuple(torch.from_numpy(np.asarray(a, dtype=np.float32)).double() for a in cots[0])
    g, gp, gvel, gc0, gom, gang = O.rollout_vjp(env, prm, st0, S, c, vel=velt, omega=omt, col=1)
    # every collider touches the blob: dropping any one of them changes the oracle's final velocities
    for drop in range(3):
        cs = [cc for k, cc in enumerate(env.colliders) if k != drop]
        e2 = dataclasses.replace(env, collider=cs[0], more=tuple(cs[1:]))
        (_, v2, _, _), _ = O.rollout(e2, prm, st0, S)
        assert np.abs(v2.numpy() - v.numpy()).max() > 1e-3, drop
    check_state(st, tuple(t.numpy() for t in (x, v, Cm, F)), "gripper actions", spec.x, S)
    check_grads(gr, tuple(t.numpy() for t in g), "gripper actions")
    ev, ec, eo = relerr(dvel, gvel.numpy()), relerr(dc0, gc0.numpy()), relerr(dom, gom.numpy())
    ea = abs(dang - float(gang)) / abs(float(gang))
    announce(f"gripper actions: dL/dvel {ev:.2e}, dL/dc0 {ec:.2e}, dL/domega {eo:.2e}, dL/dangle0 {ea:.2e}")
    assert ev < 1e-3 and ec < 1e-3 and eo < 1e-3 and ea < 1e-3


def test_collider_slots_gaps_removal_and_errors():
    # colliders in slots 0 and 2 with slot 1 empty equal the oracle's two-collider env; removing slot 2
    # (alpha 0) leaves the one-collider env; a slot outside [0, 4), an unknown shape, a motion on an
    # empty slot and a motion shorter than the rollout are refused
    import ctypes
    import dataclasses
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd._capi import MPMError
    from paper_2412_12089_amd.batch import Batch
    spec = make_env(scenes.FLUID_TAIT, N=2000, seed=190, collider=GRIP[0], v_scale=0.2)
    S = 6
    b = Batch([spec], max_substeps=S, ckpt_every=3)
    try:
        # one collider first (its launches are captured in graphs), then a second one in slot 2: the grid
        # passes must switch to the variant for several colliders
        b.set_particles_from_specs()
        b.forward(S)
        st_one = tuple(to_np(t) for t in b.get_particles(env=0))
        b.set_collider(0, GRIP[2], index=2)
        b.set_particles_from_specs()
        b.forward(S)
        st2 = tuple(to_np(t) for t in b.get_particles(env=0))
        b.set_collider(0, dataclasses.replace(GRIP[2], alpha=0.0), index=2)
        b.set_particles_from_specs()
        b.forward(S)
        st1 = tuple(to_np(t) for t in b.get_particles(env=0))
        f3 = (ctypes.c_float * 3)(0.5, 0.5, 0.5)
        for idx, shape in ((4, C.MPM_COLLIDER_BOX), (-1, C.MPM_COLLIDER_BOX), (1, 7)):
            assert b.lib.mpm_set_collider(b.h, 0, idx, shape, f3, f3, 0.05, f3, 10.0, 0.1) == C.MPM_INVALID_ARG
        with pytest.raises(MPMError):
            b.set_collider_motion(0, np.zeros((S, 3), np.float32), index=1)     # slot 1 is empty
        b.set_collider_motion(0, np.zeros((S - 2, 3), np.float32), index=0)
        b.set_particles_from_specs()
        with pytest.raises(MPMError):
            b.forward(S)
        assert b.sync(raise_on_error=False) == 0
    finally:
        b.close()
    env, prm, st0 = O.env_from_spec(spec)
    two = dataclasses.replace(env, more=(O.env_from_spec(dataclasses.replace(spec, collider=GRIP[2]))[0].collider,))
    announce("collider slots 0 and 2, then slot 2 removed")
    (x, v, Cm, F), _ = O.rollout(two, prm, st0, S)
    check_state(st2, tuple(t.numpy() for t in (x, v, Cm, F)), "slots 0 and 2", spec.x, S)
    (x, v, Cm, F), _ = O.rollout(env, prm, st0, S)
    check_state(st1, tuple(t.numpy() for t in (x, v, Cm, F)), "slot 2 removed", spec.x, S)
    check_state(st_one, tuple(t.numpy() for t in (x, v, Cm, F)), "slot 0 alone", spec.x, S)
    assert np.abs(st2[1] - st1[1]).max() > 1e-3
