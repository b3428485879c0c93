"""Scheduler logic of the continuous-batching server, on the CPU with an
executor that runs the FP64 oracle."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from oracle_executor import OracleExecutor
from paper_2412_12089_amd import scenes
from paper_2412_12089_amd.server import Server, resident_bytes


def small_requests(n=6, seed=0, N_lo=60, N_hi=160, S_lo=3, S_hi=9):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        N = int(rng.integers(N_lo, N_hi))
        mat = scenes.MIXED_MATERIALS[i % 3]
        x = scenes._f32(0.4 + rng.uniform(0, 0.15, size=(N, 3)))
        v = scenes._f32(rng.uniform(-0.5, 0.5, size=(N, 3)))
        C, F = scenes._rest_state(N)
        env = scenes.EnvSpec(n=16, dt=2e-4, rho=1e3, Vp=0.15 ** 3 / N, x=x, v=v, C=C, F=F, **mat)
        w = scenes._f32(rng.standard_normal((N, 3)))
        reqs.append(scenes.Request(i, 0.0, env, int(rng.integers(S_lo, S_hi)), bool(i % 2 == 0), w))
    return reqs


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t


def serve(reqs, n_slots=3, budget=10 ** 9, chunk=4):
    ex = OracleExecutor(n_slots, n_cap=16, N_cap=200)
    srv = Server(ex, budget, chunk=chunk, clock=FakeClock())
    done = srv.run(reqs, realtime=False)
    return srv, ex, done


def test_results_match_direct_oracle_rollouts():
    reqs = small_requests()
    srv, ex, done = serve(reqs)
    assert all(done[r.rid].status == "ok" for r in reqs)
    for r in reqs:
        env, prm, st = O.env_from_spec(r.env)
        (x, v, C, F), _ = O.rollout(env, prm, st, r.substeps)
        got = done[r.rid].state
        for a, b in zip(got, (x, v, C, F)):
            assert torch.allclose(a, b, rtol=0, atol=1e-13)
        if r.backward:
            g, gp = O.rollout_vjp(env, prm, st, r.substeps, O.linear_loss_cotangent(r.loss_weights, r.env.n_particles))
            for a, b in zip(done[r.rid].grads, g):
                assert torch.allclose(a, b, rtol=1e-10, atol=1e-12 * float(b.abs().max()))
            np.testing.assert_allclose(done[r.rid].dparams, O.param_cotangent_row(gp), rtol=1e-9, atol=1e-30)
        else:
            assert done[r.rid].grads is None


def test_work_overlaps_in_shared_calls():
    reqs = small_requests()
    srv, ex, done = serve(reqs, n_slots=3)
    assert srv.max_concurrent == 3
    # some forward call advanced more than one slot at once
    assert any(sum(1 for k in counts if k) > 1 for kind, counts in ex.calls if kind == "fwd")
    # forward and backward phases interleave across iterations
    kinds = [k for k, _ in ex.calls]
    first_rec = kinds.index("fwd_rec")
    assert "fwd" in kinds[first_rec:]


def test_tiny_budget_serialises_and_keeps_arrival_order():
    reqs = small_requests()
    biggest = max(resident_bytes(r, 4) for r in reqs)
    srv, ex, done = serve(reqs, n_slots=3, budget=biggest)
    assert all(done[r.rid].status == "ok" for r in reqs)
    assert srv.max_concurrent == 1
    adm = [done[r.rid].admitted for r in reqs]
    assert adm == sorted(adm)


def test_slots_are_reused():
    reqs = small_requests(n=7)
    srv, ex, done = serve(reqs, n_slots=2)
    assert srv.max_concurrent == 2
    assert all(done[r.rid].status == "ok" for r in reqs)
    assert sorted(srv.free) == [0, 1] and not srv.active


def test_cancel_and_reject():
    reqs = small_requests(n=4)
    ex = OracleExecutor(1, n_cap=16, N_cap=200)
    srv = Server(ex, 10 ** 9, chunk=4, clock=FakeClock())
    for r in reqs:
        srv.submit(r)
    srv.step()                      # request 0 admitted and running, others queued
    assert srv.cancel(reqs[2].rid)  # queued
    assert srv.cancel(reqs[0].rid)  # active
    while not srv.idle():
        srv.step()
    st = {rid: r.status for rid, r in srv.done.items()}
    assert st[reqs[0].rid] == "cancelled" and st[reqs[2].rid] == "cancelled"
    assert st[reqs[1].rid] == "ok" and st[reqs[3].rid] == "ok"
    big = dataclasses.replace(reqs[1], rid=99, env=dataclasses.replace(reqs[1].env, n=32))
    srv.submit(big)
    assert srv.done[99].status == "rejected"
    tiny = Server(OracleExecutor(1, n_cap=16, N_cap=200), budget_bytes=10, chunk=4, clock=FakeClock())
    tiny.submit(reqs[3])
    assert tiny.done[reqs[3].rid].status == "rejected"


def test_serving_stream_generator_is_seeded_and_shaped():
    a = scenes.serving_stream(seed=5, duration=0.2)
    b = scenes.serving_stream(seed=5, duration=0.2)
    assert [r.rid for r in a] == [r.rid for r in b] and len(a) > 10
    for r in a:
        assert r.env.n in (32, 48, 64) and 4000 <= r.env.n_particles <= 100000 and 20 <= r.substeps <= 80
        n = r.env.n
        assert (r.env.x >= (scenes.WALL + 1) / n - 1e-6).all() and (r.env.x < 1 - (scenes.WALL + 1) / n).all()
    arr = np.array([r.arrival for r in a])
    assert (np.diff(arr) > 0).all()


def test_results_can_be_dropped_for_throughput_runs():
    # keep_results=False: finished requests keep status and timing only (a long stream holds no tensors)
    reqs = small_requests(n=4)
    ex = OracleExecutor(2, n_cap=16, N_cap=200)
    srv = Server(ex, 10 ** 9, chunk=4, clock=FakeClock(), keep_results=False)
    done = srv.run(reqs, realtime=False)
    assert all(r.status == "ok" and r.state is None and r.grads is None for r in done.values())
    assert srv.stats()["ok"] == len(reqs)


def test_a_failing_request_fails_alone():
    # a request with a particle outside the valid band is reported as an error and frees its slot;
    # the others are unaffected
    reqs = small_requests(n=5)
    bad = reqs[2]
    x = bad.env.x.copy()
    x[0, 0] = 0.99
    reqs[2] = dataclasses.replace(bad, env=dataclasses.replace(bad.env, x=x))
    ex = OracleExecutor(2, n_cap=16, N_cap=200)
    srv = Server(ex, 10 ** 9, chunk=4, clock=FakeClock())
    done = srv.run(reqs, realtime=False)
    st = {rid: r for rid, r in done.items()}
    assert st[reqs[2].rid].status == "error" and st[reqs[2].rid].error & 2
    assert all(st[r.rid].status == "ok" for i, r in enumerate(reqs) if i != 2)
    assert sorted(srv.free) == [0, 1] and not srv.active
    assert srv.stats()["errors"] == 1
