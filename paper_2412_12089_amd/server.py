"""Continuous-batching rollout server over one batch of environment slots.

A request is one environment: an initial state, a material, a number of
substeps S and optionally a backward pass of L = sum_p x_p . w_p (the loss the
workloads use) back to the initial state and the parameters. The server keeps
a fixed pool of slots (environments of the batch, each with a grid and a
particle capacity) and an HBM budget for what requests keep resident:

* admission: requests queue in arrival order; the head is admitted when a
  slot is free and the bytes it keeps resident (its state, the chunk
  checkpoints a backward needs, its grid share) fit in the budget;
* every engine iteration advances every slot in its forward phase by one
  chunk of substeps in ONE batched call (slots finishing early are frozen for
  the rest of the call), and moves every slot in its backward phase one chunk
  back in ONE recorded forward + backward call: requests that arrive while
  others are running join at the next iteration, and their work shares the
  same kernel launches;
* a finished request frees its slot and its budget at once.

Per-request latency (arrival to result) and aggregate particle-substeps/s are
recorded. The executor does the arithmetic; `GPUExecutor` drives libmpmx.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from .scenes import EnvSpec, NEOHOOKEAN, Request

STATE_BYTES = 96          # x, v, C, F in FP32 per particle
GRID_NODE_BYTES = 32      # m, P, v (+ pad) per node of a slot's grid


def resident_bytes(req: Request, chunk: int) -> int:
    """Bytes a request keeps on the device while it is admitted: its state, and
    for a backward the chunk checkpoints and the cotangent it carries back."""
    N = req.env.n_particles
    nchunks = -(-req.substeps // chunk)
    ck = nchunks + 1 if req.backward else 0      # chunk checkpoints and the running cotangent
    return N * STATE_BYTES * (1 + ck) + req.env.n ** 3 * GRID_NODE_BYTES


@dataclasses.dataclass
class Result:
    rid: int
    state: tuple = None            # final (x, v, C, F)
    grads: tuple = None            # cotangents of the initial (x, v, C, F)
    dparams: np.ndarray = None     # dL/d(E, nu, rho, Vp, sigma_y, K, gamma, 0)
    arrival: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0
    status: str = "ok"             # ok / error / cancelled / rejected
    error: int = 0                 # device error bits of a failed request (1 non-finite, 2 out of the band)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class _Active:
    req: Request
    slot: int
    phase: str                     # "fwd" or "bwd"
    remaining: int
    ckpts: list
    chunk_idx: int = -1
    cot: tuple = None
    dparams: np.ndarray = None
    result: Result = None
    nbytes: int = 0


class Server:
    def __init__(self, executor, budget_bytes: int, chunk: int = 10, clock: Optional[Callable[[], float]] = None,
                 keep_results: bool = True):
        self.ex = executor
        self.keep_results = keep_results   # False: finished results keep timing and status only
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.queue: collections.deque = collections.deque()
        self.active: Dict[int, _Active] = {}
        self.free = list(range(executor.n_slots))
        self.used = 0
        self.done: Dict[int, Result] = {}
        self.clock = clock or time.perf_counter
        self.t0 = self.clock()
        self.work = 0                   # particle-substeps completed (forward + backward)
        self.iterations = 0
        self.max_concurrent = 0

    # ------------------------------------------------------------------ API
    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> int:
        n_cap, N_cap = self.ex.capacity
        if req.env.n > n_cap or req.env.n_particles > N_cap or req.substeps < 1:
            self.done[req.rid] = Result(req.rid, arrival=req.arrival, finished=self.now(), status="rejected")
            return req.rid
        if resident_bytes(req, self.chunk) > self.budget:
            self.done[req.rid] = Result(req.rid, arrival=req.arrival, finished=self.now(), status="rejected")
            return req.rid
        self.queue.append(req)
        return req.rid

    def cancel(self, rid: int) -> bool:
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                self.done[rid] = Result(rid, arrival=r.arrival, finished=self.now(), status="cancelled")
                return True
        for slot, a in list(self.active.items()):
            if a.req.rid == rid:
                self._release(slot, status="cancelled")
                return True
        return False

    def idle(self) -> bool:
        return not self.queue and not self.active

    # ------------------------------------------------------------------ engine
    def _admit(self):
        while self.queue and self.free:
            req = self.queue[0]
            need = resident_bytes(req, self.chunk)
            if self.used + need > self.budget:
                break                                    # head-of-line: arrival order is kept
            self.queue.popleft()
            slot = self.free.pop(0)
            self.ex.load(slot, req.env)
            res = Result(req.rid, arrival=req.arrival, admitted=self.now())
            self.active[slot] = _Active(req, slot, "fwd", req.substeps, [], result=res, nbytes=need)
            self.used += need
        self.max_concurrent = max(self.max_concurrent, len(self.active))

    def _release(self, slot: int, status: str = "ok"):
        a = self.active.pop(slot)
        a.result.status = status
        a.result.finished = self.now()
        if not self.keep_results:
            a.result.state = a.result.grads = a.result.dparams = None
        self.done[a.req.rid] = a.result
        self.used -= a.nbytes
        self.ex.unload(slot)
        self.free.append(slot)
        self.free.sort()

    def _forward_iteration(self):
        fwd = {s: a for s, a in self.active.items() if a.phase == "fwd"}
        if not fwd:
            return
        counts = [0] * self.ex.n_slots
        for s, a in fwd.items():
            counts[s] = min(self.chunk, a.remaining)
            if a.req.backward:
                a.ckpts.append((self.ex.snapshot(s), counts[s]))
        self.ex.forward(counts, record=False)
        finished = []
        for s, a in fwd.items():
            a.remaining -= counts[s]
            self.work += a.req.env.n_particles * counts[s]
            if a.remaining == 0:
                finished.append(s)
        if finished:
            for s in finished:
                a = self.active[s]
                a.result.state = self.ex.read(s)
                if a.req.backward:
                    a.phase = "bwd"
                    a.chunk_idx = len(a.ckpts) - 1
                    a.cot = self.ex.loss_cotangent(a.req)
                    a.dparams = np.zeros(8)
            self._sync()
            for s in finished:
                if s in self.active and not self.active[s].req.backward:
                    self._release(s)

    def _backward_iteration(self):
        bwd = {s: a for s, a in self.active.items() if a.phase == "bwd"}
        if not bwd:
            return
        counts = [0] * self.ex.n_slots
        for s, a in bwd.items():
            snap, k = a.ckpts[a.chunk_idx]
            self.ex.restore(s, snap)
            counts[s] = k
        self.ex.forward(counts, record=True)
        out = self.ex.backward({s: a.cot for s, a in bwd.items()})
        finished = []
        for s, a in bwd.items():
            g, dp = out[s]
            a.cot = g
            a.dparams = a.dparams + dp
            self.work += a.req.env.n_particles * counts[s]
            a.ckpts[a.chunk_idx] = None                  # its memory can go
            a.chunk_idx -= 1
            if a.chunk_idx < 0:
                finished.append(s)
        if finished:
            for s in finished:
                a = self.active[s]
                a.result.grads = a.cot
                a.result.dparams = a.dparams
            self._sync()
            for s in finished:
                if s in self.active:
                    self._release(s)

    def _sync(self):
        """Wait for the device; a request whose environment reported an error
        (non-finite state, a particle out of the band) fails alone and frees its slot."""
        for slot, bits in (self.ex.sync() or {}).items():
            if slot in self.active and bits:
                self.active[slot].result.error = int(bits)
                self._release(slot, status="error")

    def step(self) -> None:
        """One engine iteration: admit, one forward chunk, one backward chunk."""
        self._admit()
        self._forward_iteration()
        self._backward_iteration()
        self.iterations += 1

    def run(self, requests: List[Request], realtime: bool = True, timeout_s: float = 600.0) -> Dict[int, Result]:
        """Feed `requests` by their arrival times (seconds from now) and serve until all are done.

        With realtime=False arrivals are released as soon as the engine is
        idle or reaches their time on the engine's own clock (for tests)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = self.clock()
        start = self.t0
        while pending or not self.idle():
            now = self.now()
            while pending and (pending[0].arrival <= now or (not realtime and self.idle())):
                r = pending.popleft()
                if not realtime and r.arrival > now:
                    r = dataclasses.replace(r, arrival=now)
                self.submit(r)
            if self.idle():
                if pending and realtime:
                    time.sleep(max(0.0, min(pending[0].arrival - self.now(), 0.01)))
                continue
            self.step()
            if self.clock() - start > timeout_s:
                raise TimeoutError("server did not drain in time")
        self._sync()
        return self.done

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.done.values() if r.status == "ok"])
        errors = int(sum(r.status == "error" for r in self.done.values()))
        span = max((r.finished for r in self.done.values()), default=0.0)
        return {
            "requests": len(self.done),
            "ok": int(sum(r.status == "ok" for r in self.done.values())),
            "errors": errors,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "particle_substeps_per_s": self.work / span if span > 0 else None,
            "iterations": self.iterations,
            "max_concurrent": self.max_concurrent,
            "wall_s": span,
        }


class GPUExecutor:
    """Slots = environments of one libmpmx batch (capacity n_cap^3 grid, N_cap particles)."""

    def __init__(self, n_slots: int, n_cap: int = 64, N_cap: int = 100_000, chunk: int = 10, device=None):
        import torch
        from .batch import Batch
        self.torch = torch
        self.n_slots = n_slots
        self.capacity = (n_cap, N_cap)
        self.chunk = chunk
        protos = []
        for _ in range(n_slots):
            protos.append(EnvSpec(n=n_cap, dt=5e-5, material=NEOHOOKEAN, E=1e3, nu=0.3, rho=1e3, Vp=1e-6,
                                  x=np.zeros((N_cap, 3), np.float32)))
        self.batch = Batch(protos, max_substeps=chunk, ckpt_every=chunk, mode="batched", device=device)
        self.device = self.batch.device
        for i in range(n_slots):
            self.unload(i)

    def _empty(self):
        return EnvSpec(n=self.capacity[0], dt=5e-5, material=NEOHOOKEAN, E=1e3, nu=0.3, rho=1e3, Vp=1e-6,
                       x=np.zeros((0, 3), np.float32))

    def load(self, slot: int, spec: EnvSpec):
        t = self.torch
        self.batch.configure_env(slot, spec)
        self.batch.set_particles(*(t.from_numpy(getattr(spec, k)) for k in ("x", "v", "C", "F")), env=slot)

    def unload(self, slot: int):
        self.batch.configure_env(slot, self._empty())

    def snapshot(self, slot: int):
        return self.batch.get_particles(env=slot)

    def restore(self, slot: int, snap):
        self.batch.set_particles(*snap, env=slot)

    def forward(self, counts, record: bool):
        self.batch.forward_envs(counts, record=record)

    def loss_cotangent(self, req: Request):
        t = self.torch
        N = req.env.n_particles
        z3 = t.zeros(N, 3, device=self.device)
        z33 = t.zeros(N, 3, 3, device=self.device)
        return (t.from_numpy(req.loss_weights).to(self.device), z3, z33, z33.clone())

    def backward(self, cots: Dict[int, tuple]):
        t = self.torch
        b = self.batch
        parts = [[], [], [], []]
        for s in range(self.n_slots):
            n = b.counts[s]
            if n == 0:
                continue
            c = cots.get(s)
            shapes = ((n, 3), (n, 3), (n, 3, 3), (n, 3, 3))
            for k in range(4):
                parts[k].append(c[k] if c is not None else t.zeros(*shapes[k], device=self.device))
        cat = [t.cat(p, 0) if p else None for p in parts]
        dx, dv, dC, dF, dp = b.backward(*cat)
        out = {}
        for s in cots:
            lo, hi = int(b.offsets[s]), int(b.offsets[s + 1])
            # copies: a view would keep the whole batch-wide output alive as long as the request does
            out[s] = ((dx[lo:hi].clone(), dv[lo:hi].clone(), dC[lo:hi].clone(), dF[lo:hi].clone()),
                      dp[s].cpu().numpy())
        return out

    def read(self, slot: int):
        return self.batch.get_particles(env=slot)

    def sync(self):
        """Waits for the device; returns {slot: error bits} for slots that reported errors since the last call."""
        self.batch.sync(raise_on_error=False)
        errs = self.batch.env_errors()
        return {i: int(b) for i, b in enumerate(errs) if b}

    def close(self):
        self.batch.close()
