"""Host logic of the library's continuous-batching server, on the CPU: the
server in its dry mode schedules exactly as on the device (admission by budget
in arrival order, one forward chunk per step for requests in their forward
phase, one backward chunk per step for those in their backward phase, slot
reuse, cancel, reject) without device work. The numerics of served requests
are checked on the GPU (tests/test_gpu_server.py)."""
import ctypes

import numpy as np
import pytest

from paper_2412_12089_amd import _capi as C
from paper_2412_12089_amd import scenes
from paper_2412_12089_amd.server import Server


def req(rid, N=1000, n=32, S=10, backward=False, material=scenes.NEOHOOKEAN):
    x = np.zeros((N, 3), np.float32)
    env = scenes.EnvSpec(n=n, dt=5e-5, material=material, E=5e3, nu=0.3, rho=1e3, Vp=1e-6, x=x)
    return scenes.Request(rid, 0.0, env, S, backward, np.zeros((N, 3), np.float32))


def resident(r, chunk):
    """Device bytes the library reserves for an admitted request."""
    N, n = r.env.n_particles, r.env.n
    b = 96 * N + 32 * n ** 3
    if r.backward:
        b += -(-r.substeps // chunk) * 25 * 4 * N + 96 * N
    return b


def state(srv, sid):
    st = C.mpm_request_status()
    assert srv.lib.mpm_server_poll(srv.h, sid, ctypes.byref(st)) == 0
    return st.state


def dry(n_slots=2, chunk=4, budget=1 << 40, n_cap=64, N_cap=100_000):
    return Server(n_slots, n_cap, N_cap, chunk, budget, dry=True)


def test_steps_to_finish_follow_the_chunks():
    # S = 10, chunk 4: forward chunks at steps 1, 2, 3; the backward starts in the step whose forward
    # ends and undoes one chunk per step (3 chunks: steps 3, 4, 5)
    srv = dry(n_slots=2, chunk=4)
    a = srv.submit(req(0, S=10, backward=False))
    b = srv.submit(req(1, S=10, backward=True))
    finished = {}
    for step in range(1, 8):
        srv.lib.mpm_server_step(srv.h)
        for sid in (a, b):
            if sid not in finished:
                s = state(srv, sid)
                if s == C.MPM_REQ_DONE:
                    finished[sid] = step
                else:
                    assert s == C.MPM_REQ_RUNNING
    assert finished == {a: 3, b: 5}
    assert state(srv, a) == C.MPM_REQ_UNKNOWN     # a final state is reported once
    st = srv.stats()
    assert st["ok"] == 2 and st["particle_substeps"] == 2 * 1000 * 10   # N S once per request
    assert st["steps"] == 7 and st["max_concurrent"] == 2
    srv.close()


def test_admission_by_budget_keeps_arrival_order():
    chunk = 5
    big, small = req(0, N=50_000, S=10), req(2, N=2000, S=5)
    big2 = req(1, N=50_000, S=10)
    budget = resident(big, chunk) + resident(small, chunk) - 1   # big + small do not fit together
    srv = dry(n_slots=4, chunk=chunk, budget=budget)
    ids = [srv.submit(r) for r in (big, big2, small)]
    srv.lib.mpm_server_step(srv.h)
    # the second big request waits for the budget, and the small one behind it is not admitted first
    assert [state(srv, i) for i in ids] == [C.MPM_REQ_RUNNING, C.MPM_REQ_QUEUED, C.MPM_REQ_QUEUED]
    assert srv.stats()["bytes_in_use"] == resident(big, chunk)
    srv.lib.mpm_server_step(srv.h)          # big finishes (2 chunks) and frees its budget
    assert state(srv, ids[0]) == C.MPM_REQ_DONE
    srv.lib.mpm_server_step(srv.h)          # big2 admitted; small does not fit beside it
    assert state(srv, ids[1]) == C.MPM_REQ_RUNNING and state(srv, ids[2]) == C.MPM_REQ_QUEUED
    for _ in range(4):
        srv.lib.mpm_server_step(srv.h)
    srv.collect()
    assert srv.stats()["ok"] == 3 and srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_budget_boundary_and_capacity_rejects():
    chunk = 4
    r = req(0, N=3000, S=9, backward=True)
    exact = resident(r, chunk)
    srv = dry(chunk=chunk, budget=exact)
    ok = srv.submit(r)
    too_big = srv.submit(req(1, N=3001, S=9, backward=True))       # one particle more than the budget holds
    grid = srv.submit(req(2, n=96))                                 # grid above the slot capacity (64)
    parts = srv.submit(req(3, N=100_001))                           # particles above the slot capacity
    for sid in (too_big, grid, parts):
        assert state(srv, sid) == C.MPM_REQ_REJECTED
    srv.lib.mpm_server_step(srv.h)
    assert state(srv, ok) == C.MPM_REQ_RUNNING
    assert srv.stats()["rejected"] == 3
    srv.close()


def test_cancel_frees_the_slot_and_budget():
    srv = dry(n_slots=1, chunk=2)
    a = srv.submit(req(0, S=8))
    b = srv.submit(req(1, S=2))
    c = srv.submit(req(2, S=2))
    srv.lib.mpm_server_step(srv.h)
    assert state(srv, a) == C.MPM_REQ_RUNNING and state(srv, b) == C.MPM_REQ_QUEUED
    assert srv.lib.mpm_server_cancel(srv.h, c) == 0                 # queued
    assert srv.lib.mpm_server_cancel(srv.h, a) == 0                 # running: slot and budget free at once
    assert srv.stats()["bytes_in_use"] == 0
    assert state(srv, a) == C.MPM_REQ_CANCELLED and state(srv, c) == C.MPM_REQ_CANCELLED
    assert srv.lib.mpm_server_cancel(srv.h, a) == C.MPM_INVALID_ARG  # already final (and polled)
    srv.lib.mpm_server_step(srv.h)
    assert state(srv, b) == C.MPM_REQ_DONE
    st = srv.stats()
    assert st["cancelled"] == 2 and st["ok"] == 1
    srv.close()


def test_slots_are_reused_in_order():
    srv = dry(n_slots=2, chunk=10)
    reqs = [req(i, S=10 * (1 + i % 3)) for i in range(7)]
    done = srv.run(reqs, realtime=False)
    assert sorted(done) == list(range(7))
    assert all(r.status == "ok" for r in done.values())
    st = srv.stats()
    assert st["max_concurrent"] == 2 and st["running"] == 0 and st["queued"] == 0
    assert st["particle_substeps"] == sum(r.env.n_particles * r.substeps for r in reqs)
    srv.close()


def test_invalid_requests_are_refused():
    srv = dry()
    lib = srv.lib
    r = C.mpm_request()
    r.env.n, r.env.material, r.env.n_particles, r.env.dt, r.env.wall = 32, 0, 10, 5e-5, 3
    r.params[1] = 0.3
    sid = ctypes.c_int64()
    r.substeps = 5
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG   # null arrays
    keep = np.zeros(4, np.float32)
    r.x = r.v = r.C = r.F = keep.ctypes.data
    r.substeps = 0
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG   # S < 1
    r.substeps = 5
    r.params[1] = 0.5
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG   # nu
    r.params[1] = 0.3
    r.env.material = 9
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG
    r.env.material = 0
    r.n_more = C.MPM_MAX_COLLIDERS                                                                   # too many
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG
    r.n_more = 1
    r.more[0].shape = 5                                                                              # no shape
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_INVALID_ARG
    r.more[0].shape = C.MPM_COLLIDER_SPHERE
    assert lib.mpm_server_submit(srv.h, ctypes.byref(r), ctypes.byref(sid)) == C.MPM_OK
    assert lib.mpm_server_cancel(srv.h, 12345) == C.MPM_INVALID_ARG
    st = C.mpm_request_status()
    assert lib.mpm_server_poll(srv.h, 12345, ctypes.byref(st)) == 0 and st.state == C.MPM_REQ_UNKNOWN
    srv.close()


@pytest.mark.parametrize("kw", [dict(n_slots=0), dict(n_cap=30), dict(N_cap=0), dict(chunk=0), dict(budget=-1)])
def test_create_rejects_bad_descriptions(kw):
    args = dict(n_slots=2, n_cap=32, N_cap=100, chunk=4, budget=1 << 20)
    args.update(kw)
    with pytest.raises(C.MPMError):
        Server(args["n_slots"], args["n_cap"], args["N_cap"], args["chunk"], args["budget"], dry=True)


def test_latency_is_counted_from_the_stated_arrival():
    import time
    srv = dry(n_slots=1, chunk=4)
    time.sleep(0.6)
    t = srv.now()
    a = srv.submit(req(0, S=4), arrival=t - 0.5)   # arrived half a second before it was submitted
    srv.step()
    r = srv.done[0]
    assert r.status == "ok" and r.latency >= 0.5 and abs(r.arrival - (t - 0.5)) < 1e-9
    srv.close()
