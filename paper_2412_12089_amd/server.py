"""Python driver of the library's continuous-batching server (``mpm_server_*``
in include/mpm.h).

Argument marshalling only. The scheduling (admission by HBM budget in arrival
order, slots of one batch, one batched forward chunk and one batched backward
chunk per engine step), the chunk checkpoints, the running cotangents and the
FP64 sums of the parameter cotangents all live in the library. This module
turns requests into device tensors, keeps them alive until the library reports
the request finished, and feeds a stream of requests by their arrival times.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import _capi as C
from .scenes import Request


@dataclasses.dataclass
class Result:
    rid: int
    status: str = "ok"            # ok / error / cancelled / rejected
    state: tuple = None           # final (x, v, C, F), device tensors
    grads: tuple = None           # cotangents of the initial (x, v, C, F)
    dparams: np.ndarray = None    # dL/d(E, nu, rho, Vp, sigma_y, K, gamma, 0)
    arrival: float = 0.0          # server-clock seconds
    admitted: float = 0.0
    finished: float = 0.0
    error: int = 0                # device error bits (1 non-finite, 2 out of the band)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """A server of `n_slots` slots (grid capacity n_cap^3, N_cap particles each).

    keep_results=False: finished requests keep status and timing only (no
    output tensors are allocated), for long throughput runs. dry=True: the
    library schedules without device work (host-logic tests)."""

    def __init__(self, n_slots: int, n_cap: int, N_cap: int, chunk: int, budget_bytes: int, device=None,
                 keep_results: bool = True, dry: bool = False):
        self.lib = C.load()
        self.dry = dry
        self.keep_results = keep_results and not dry
        self.device = None
        self.allocator = None
        stream = None
        if not dry:
            import torch
            from .batch import TorchAllocator
            self.torch = torch
            self.device = torch.device(device or "cuda")
            self.allocator = TorchAllocator(self.device)
            stream = torch.cuda.current_stream(self.device)
        d = C.mpm_server_desc(int(n_slots), int(n_cap), int(N_cap), int(chunk), C.MPM_SERVER_DRY if dry else 0,
                              int(budget_bytes))
        h = ctypes.c_void_p()
        alloc = ctypes.byref(self.allocator.struct) if self.allocator else None
        if dry:
            self._chk(self.lib.mpm_server_create(ctypes.byref(d), None, None, ctypes.byref(h)), "mpm_server_create")
        else:
            with self.torch.cuda.device(self.device):
                self._chk(self.lib.mpm_server_create(ctypes.byref(d), alloc, ctypes.c_void_p(stream.cuda_stream),
                                                     ctypes.byref(h)), "mpm_server_create")
        self.h = h
        self.n_slots, self.chunk = n_slots, chunk
        self.live: Dict[int, tuple] = {}       # library id -> (request, tensors kept alive, outputs)
        self.done: Dict[int, Result] = {}      # request rid -> result
        self._dummy = np.zeros(4, np.float32)  # dry mode: a non-null host address for the state arrays

    def _chk(self, code, where):
        return C.check(code, where, getattr(self, "h", None), server=True)

    # ------------------------------------------------------------------ API
    def now(self) -> float:
        return float(self.lib.mpm_server_now(self.h))

    def submit(self, req: Request, arrival: Optional[float] = None) -> int:
        """Queues `req`; arrival: server-clock seconds (None = now). Returns the library id."""
        e = req.env
        r = C.mpm_request()
        r.env.n, r.env.material, r.env.n_particles, r.env.dt, r.env.wall = e.n, e.material, e.n_particles, e.dt, e.wall
        r.env.gravity[:] = list(e.gravity)
        r.params[:] = [float(v) for v in e.params()]
        r.substeps, r.backward = int(req.substeps), int(bool(req.backward))
        r.arrival = -1.0 if arrival is None else float(arrival)
        if e.collider is not None:
            c = e.collider
            r.has_collider = 2 if getattr(c, "shape", "box") == "sphere" else (
                3 if getattr(c, "rounding", 0.0) > 0.0 else 1)
            r.c_round = float(getattr(c, "rounding", 0.0))
            r.c_center[:], r.c_half[:], r.c_vel[:] = list(c.center), list(c.half), list(c.velocity)
            r.c_alpha, r.c_mu = float(c.alpha), float(c.mu_b)
        more = list(getattr(e, "more_colliders", ()))
        if len(more) > C.MPM_MAX_COLLIDERS - 1:
            raise ValueError(f"at most {C.MPM_MAX_COLLIDERS - 1} further colliders per request")
        r.n_more = len(more)
        for k, c in enumerate(more):
            if c.rotates:
                raise ValueError("served requests take colliders that translate only")
            m = r.more[k]
            sphere = getattr(c, "shape", "box") == "sphere"
            rounding = float(getattr(c, "rounding", 0.0))
            m.shape = (C.MPM_COLLIDER_SPHERE if sphere else
                       C.MPM_COLLIDER_ROUNDED_BOX if rounding > 0.0 else C.MPM_COLLIDER_BOX)
            m.radius = float(c.half[0]) if sphere else rounding
            m.center[:], m.half[:], m.vel[:] = list(c.center), list(c.half), list(c.velocity)
            m.alpha, m.mu_b = float(c.alpha), float(c.mu_b)
        keep, outs = [], None
        if self.dry:
            addr = self._dummy.ctypes.data
            r.x = r.v = r.C = r.F = addr
        else:
            t = self.torch
            dev = lambda a: t.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)
            ins = [dev(getattr(e, k)) for k in ("x", "v", "C", "F")]
            keep += ins
            r.x, r.v, r.C, r.F = (C.ptr(a) for a in ins)
            N = e.n_particles
            if req.backward:
                gx = dev(req.loss_weights)   # L = sum_p x_p . w_p: only x has a cotangent
                keep.append(gx)
                r.gx = C.ptr(gx)
            if self.keep_results:
                st = (t.empty(N, 3, device=self.device), t.empty(N, 3, device=self.device),
                      t.empty(N, 3, 3, device=self.device), t.empty(N, 3, 3, device=self.device))
                r.out_x, r.out_v, r.out_C, r.out_F = (C.ptr(a) for a in st)
                gr = None
                if req.backward:
                    gr = tuple(t.empty_like(a) for a in st)
                    r.dx0, r.dv0, r.dC0, r.dF0 = (C.ptr(a) for a in gr)
                outs = (st, gr)
        sid = ctypes.c_int64()
        self._chk(self.lib.mpm_server_submit(self.h, ctypes.byref(r), ctypes.byref(sid)), "mpm_server_submit")
        self.live[sid.value] = (req, keep, outs)
        return sid.value

    def step(self) -> None:
        """One engine step of the library, then collect finished requests."""
        self._chk(self.lib.mpm_server_step(self.h), "mpm_server_step")
        self.collect()

    def collect(self) -> None:
        st = C.mpm_request_status()
        for sid in list(self.live):
            self._chk(self.lib.mpm_server_poll(self.h, sid, ctypes.byref(st)), "mpm_server_poll")
            if st.state in (C.MPM_REQ_QUEUED, C.MPM_REQ_RUNNING):
                continue
            req, _, outs = self.live.pop(sid)
            res = Result(req.rid, status=C.REQ_STATE_NAMES[st.state], arrival=st.arrival, admitted=st.admitted,
                         finished=st.finished, error=int(st.error_bits))
            if st.state == C.MPM_REQ_DONE:
                res.dparams = np.array(st.dparams[:], dtype=np.float64) if req.backward else None
                if outs is not None:
                    res.state = outs[0]
                    res.grads = outs[1]
            self.done[req.rid] = res

    def cancel(self, sid: int) -> None:
        self._chk(self.lib.mpm_server_cancel(self.h, int(sid)), "mpm_server_cancel")
        self.collect()

    def idle(self) -> bool:
        return bool(self.lib.mpm_server_idle(self.h))

    def run(self, requests: List[Request], realtime: bool = True, timeout_s: float = 600.0) -> Dict[int, Result]:
        """Serves `requests` until all are finished. realtime=True: each is
        submitted when the server clock reaches its arrival (seconds from the
        start of this call) and stamped with that arrival, so queueing behind
        a running engine step counts in its latency; realtime=False: all are
        submitted at once."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = self.now()
        while pending or not self.idle() or self.live:
            now = self.now()
            while pending and (not realtime or t0 + pending[0].arrival <= now):
                r = pending.popleft()
                self.submit(r, arrival=(t0 + r.arrival) if realtime else None)
            if self.idle():
                self.collect()
                if pending and realtime:
                    time.sleep(max(0.0, min(t0 + pending[0].arrival - self.now(), 0.01)))
                continue
            self.step()
            if self.now() - t0 > timeout_s:
                raise TimeoutError("server did not drain in time")
        return self.done

    def stats(self) -> dict:
        s = C.mpm_server_stats()
        self._chk(self.lib.mpm_server_stats_get(self.h, ctypes.byref(s)), "mpm_server_stats_get")
        span = s.last_finish - s.first_arrival
        return {
            "requests": int(s.submitted), "ok": int(s.done), "errors": int(s.errors), "cancelled": int(s.cancelled),
            "rejected": int(s.rejected), "queued": int(s.queued), "running": int(s.running),
            "p50_ms": float(s.p50_ms) if s.done else None, "p99_ms": float(s.p99_ms) if s.done else None,
            # each finished request's N S counted once, with or without a backward
            "particle_substeps": int(s.particle_substeps),
            "particle_substeps_per_s": s.particle_substeps / span if span > 0 else None,
            "steps": int(s.steps), "max_concurrent": int(s.max_running), "bytes_in_use": int(s.bytes_in_use),
            "wall_s": span,
        }

    def close(self) -> None:
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mpm_server_destroy(self.h)
            self.h = None
        self.live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
