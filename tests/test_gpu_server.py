"""The continuous-batching server on the GPU: each request's result is the
same alone and in the mix (and matches the oracle)."""
import dataclasses

import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import oracle_rollout, relerr
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


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
        env = scenes.EnvSpec(n=grid, dt=5e-5, rho=1e3, Vp=side ** 3 / N, x=x, v=v, C=C, F=F, **mat)
        w = scenes._f32(rng.standard_normal((N, 3)))
        out.append(scenes.Request(i, 0.0, env, int(rng.integers(12, 26)), bool(i % 2 == 0), w))
    return out


def serve(reqs, n_slots, chunk=5):
    from paper_2412_12089_amd.server import GPUExecutor, Server
    ex = GPUExecutor(n_slots, n_cap=48, N_cap=6000, chunk=chunk)
    srv = Server(ex, budget_bytes=8 << 30, chunk=chunk)
    done = srv.run(reqs, realtime=False)
    out = {}
    for rid, r in done.items():
        out[rid] = dict(status=r.status,
                        state=None if r.state is None else [t.cpu().double().numpy() for t in r.state],
                        grads=None if r.grads is None else [t.cpu().double().numpy() for t in r.grads],
                        dparams=r.dparams)
    stats = srv.stats()
    ex.close()
    return out, stats


def test_each_request_is_the_same_alone_and_in_the_mix():
    reqs = requests()
    print(f"[gpu-test] server: {len(reqs)} requests on 4 slots", flush=True)
    mix, stats = serve(reqs, n_slots=4)
    assert stats["max_concurrent"] == 4
    for r in reqs:
        print(f"[gpu-test] request {r.rid} alone", flush=True)
        alone, _ = serve([dataclasses.replace(r)], n_slots=1)
        a, m = alone[r.rid], mix[r.rid]
        assert a["status"] == m["status"] == "ok"
        for j in range(4):
            assert relerr(m["state"][j], a["state"][j]) < 1e-5, (r.rid, j)
        if r.backward:
            for j in range(4):
                assert relerr(m["grads"][j], a["grads"][j]) < 1e-4, (r.rid, j)
            sel = [0, 1, 4, 5, 6]
            np.testing.assert_allclose(m["dparams"][sel], a["dparams"][sel], rtol=1e-4, atol=1e-30)
    # two requests (one with a backward) against the oracle
    for r in (reqs[0], reqs[1]):
        cot = None
        if r.backward:
            N = r.env.n_particles
            cot = (r.loss_weights, np.zeros((N, 3), np.float32), np.zeros((N, 3, 3), np.float32),
                   np.zeros((N, 3, 3), np.float32))
        o = oracle_rollout(r.env, r.substeps, cot)
        for j in range(2):
            assert relerr(mix[r.rid]["state"][j], o["state"][j]) < 1e-5
        if cot is not None:
            for j in range(4):
                assert relerr(mix[r.rid]["grads"][j], o["grads"][j]) < 1e-3


def test_a_failing_request_fails_alone_on_the_device():
    # one request has a particle outside the valid band: the device error word fails it alone
    reqs = requests(n=4, seed=12)
    x = reqs[1].env.x.copy()
    x[0] = (0.995, 0.5, 0.5)
    reqs[1] = dataclasses.replace(reqs[1], env=dataclasses.replace(reqs[1].env, x=x))
    print("[gpu-test] server with one out-of-band request", flush=True)
    out, stats = serve(reqs, n_slots=2)
    assert out[reqs[1].rid]["status"] == "error"
    assert all(out[r.rid]["status"] == "ok" for i, r in enumerate(reqs) if i != 1)
    assert stats["errors"] == 1
