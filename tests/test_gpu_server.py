"""The library's continuous-batching server on the GPU: each request's result
is the same alone and in the mix, and matches the oracle -- including an
80-substep backward (8 chunks, each recomputed from its checkpoint) with the
parameter cotangents, a request whose box collider moves, whose clock must
follow it through its chunks while other slots are loaded and restored, and a
request with two colliders (a ball and a plate)."""
import dataclasses

import numpy as np
import pytest

from conftest import gpu_available
from gpu_util import assert_grads, assert_params, assert_state, oracle_rollout, relerr
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def announce(msg):
    print(f"[gpu-server] {msg}", flush=True)


def requests(n=8, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.integers(2000, 6000))
        grid = (32, 48)[i % 2]
        mat = dict(scenes.MIXED_MATERIALS[i % 3])
        if mat["material"] == scenes.VONMISES:
            mat["sigma_y"] = 5.0
        side = 0.18
        lo = rng.uniform(0.3, 0.5, size=3)
        x = scenes._f32(lo + rng.uniform(0, side, size=(N, 3)))
        v = scenes._f32(rng.uniform(-0.5, 0.5, size=(N, 3)))
        C, F = scenes._rest_state(N)
        collider, more = None, ()
        if i == 3:   # a box moving into the particles
            collider = scenes.BoxCollider(center=(float(lo[0]) + side + 0.03, 0.5, 0.5), half=(0.02, 0.3, 0.3),
                                          velocity=(-0.6, 0.0, 0.0), alpha=2.0 * grid, mu_b=0.5)
        if i == 6:   # a ball moving into the particles
            collider = scenes.sphere_collider(center=(float(lo[0]) + side + 0.04, float(lo[1]) + 0.09,
                                                      float(lo[2]) + 0.09), radius=0.06, velocity=(-0.6, 0.0, 0.0),
                                              alpha=2.0 * grid, mu_b=0.5)
            # and a second collider, a plate pushing from the other side
            more = (scenes.BoxCollider(center=(float(lo[0]) - 0.03, 0.5, 0.5), half=(0.02, 0.3, 0.3),
                                       velocity=(0.5, 0.0, 0.0), alpha=2.0 * grid, mu_b=0.3),)
        env = scenes.EnvSpec(n=grid, dt=5e-5, rho=1e3, Vp=side ** 3 / N, x=x, v=v, C=C, F=F, collider=collider,
                             more_colliders=more, **mat)
        w = scenes._f32(rng.standard_normal((N, 3)))
        S = 80 if i == 0 else int(rng.integers(12, 36))
        out.append(scenes.Request(i, 0.0, env, S, bool(i % 2 == 0) or i == 3, w))
    return out


def serve(reqs, n_slots, chunk=10):
    from paper_2412_12089_amd.server import Server
    srv = Server(n_slots, n_cap=48, N_cap=6000, chunk=chunk, budget_bytes=8 << 30)
    done = srv.run(reqs, realtime=False)
    out = {}
    for rid, r in done.items():
        out[rid] = dict(status=r.status,
                        state=None if r.state is None else [t.cpu().double().numpy() for t in r.state],
                        grads=None if r.grads is None else [t.cpu().double().numpy() for t in r.grads],
                        dparams=r.dparams)
    stats = srv.stats()
    srv.close()
    return out, stats


def loss_cot(r):
    N = r.env.n_particles
    return (r.loss_weights, np.zeros((N, 3), np.float32), np.zeros((N, 3, 3), np.float32),
            np.zeros((N, 3, 3), np.float32))


def test_each_request_is_the_same_alone_and_in_the_mix():
    reqs = requests()
    announce(f"{len(reqs)} requests on 4 slots (chunk 10)")
    mix, stats = serve(reqs, n_slots=4)
    assert stats["max_concurrent"] == 4 and stats["ok"] == len(reqs)
    assert stats["particle_substeps"] == sum(r.env.n_particles * r.substeps for r in reqs)
    for r in reqs:
        alone, _ = serve([dataclasses.replace(r)], n_slots=1)
        a, m = alone[r.rid], mix[r.rid]
        assert a["status"] == m["status"] == "ok"
        es = max(relerr(m["state"][j], a["state"][j]) for j in range(4))
        eg = max(relerr(m["grads"][j], a["grads"][j]) for j in range(4)) if r.backward else 0.0
        announce(f"request {r.rid} (S={r.substeps}, backward={r.backward}) mix vs alone: state {es:.1e} grads {eg:.1e}")
        assert es < 1e-5 and eg < 1e-4
        if r.backward:
            np.testing.assert_allclose(m["dparams"][[0, 1, 2, 4, 5, 6]], a["dparams"][[0, 1, 2, 4, 5, 6]],
                                       rtol=1e-4, atol=1e-30)
            assert m["dparams"][3] == 0.0 and a["dparams"][3] == 0.0
    # against the oracle: the 80-substep backward (8 chunks), the moving box, the moving ball, a forward-only request
    for r in (reqs[0], reqs[3], reqs[6], reqs[1]):
        cot = loss_cot(r) if r.backward else None
        o = oracle_rollout(r.env, r.substeps, cot)
        tag = f"served request {r.rid} (S={r.substeps}{', moving ' + r.env.collider.shape if r.env.collider else ''})"
        assert_state(mix[r.rid]["state"], o["state"], r.env.x, tag, announce, S=r.substeps)
        if cot is not None:
            assert_grads(mix[r.rid]["grads"], o["grads"], tag, announce)
            pidx = {scenes.NEOHOOKEAN: (0, 1), scenes.VONMISES: (0, 1, 4), scenes.FLUID_TAIT: (5, 6)}[r.env.material]
            assert_params(mix[r.rid]["dparams"], o["dparams"], pidx + (2, 3), tag, r.env.params(), announce)


def test_a_failing_request_fails_alone_on_the_device():
    # one request has a particle outside the valid band: the device error word fails it alone
    reqs = requests(n=4, seed=12)
    x = reqs[1].env.x.copy()
    x[0] = (0.995, 0.5, 0.5)
    reqs[1] = dataclasses.replace(reqs[1], env=dataclasses.replace(reqs[1].env, x=x))
    announce("server with one out-of-band request")
    out, stats = serve(reqs, n_slots=2)
    assert out[reqs[1].rid]["status"] == "error"
    assert all(out[r.rid]["status"] == "ok" for i, r in enumerate(reqs) if i != 1)
    assert stats["errors"] == 1
