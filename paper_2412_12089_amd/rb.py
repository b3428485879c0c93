"""Python binding of the rigid-body batch (include/mpm_rb.h): argument marshalling only.

`RbBatch` owns a library handle and passes torch CUDA tensors by address;
every step runs in the library's HIP kernels. `RBRollout` makes a recorded
forward and its adjoint an autograd Function, differentiable in the initial
state, the torques and the per-env parameters; calls on one batch can be
chained (a backward whose record was replaced re-runs its forward first).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _capi as C


def _f32(t, device) -> torch.Tensor:
    return torch.as_tensor(t, dtype=torch.float32, device=device).contiguous()


def pack_links(links: Sequence) -> tuple:
    """C arrays of links and contact spheres from objects with the fields of
    `rb_scenes.RbLink` (parent, joint_rot [3, 3], joint_pos, axis, mass, com,
    inertia [3, 3] about the COM, contacts [(centre, radius)], and optionally
    joint = "revolute" | "prismatic"))."""
    n = len(links)
    L = (C.mpm_rb_link * n)()
    cts = []
    for i, k in enumerate(links):
        L[i].parent = int(k.parent)
        L[i].joint_rot[:] = [float(v) for v in np.asarray(k.joint_rot, dtype=np.float64).reshape(9)]
        L[i].joint_pos[:] = [float(v) for v in np.asarray(k.joint_pos, dtype=np.float64)]
        L[i].axis[:] = [float(v) for v in np.asarray(k.axis, dtype=np.float64)]
        L[i].mass = float(k.mass)
        L[i].com[:] = [float(v) for v in np.asarray(k.com, dtype=np.float64)]
        I = np.asarray(k.inertia, dtype=np.float64)
        L[i].inertia[:] = [I[0, 0], I[1, 1], I[2, 2], I[0, 1], I[0, 2], I[1, 2]]
        kind = getattr(k, "joint", "revolute")
        if kind not in ("revolute", "prismatic"):
            raise ValueError(f"link {i}: unknown joint kind {kind!r}")
        L[i].joint = C.MPM_RB_PRISMATIC if kind == "prismatic" else C.MPM_RB_REVOLUTE
        for (c, r) in k.contacts:
            cts.append((i, np.asarray(c, dtype=np.float64), float(r)))
    K = (C.mpm_rb_contact * max(len(cts), 1))()
    for j, (i, c, r) in enumerate(cts):
        K[j].link = i
        K[j].centre[:] = [float(v) for v in c]
        K[j].radius = r
    return L, K, len(cts)


class RbBatch:
    """E articulated bodies sharing one link tree."""

    def __init__(self, links: Sequence, n_envs: int, max_substeps: int, dt: float, gravity=(0.0, 0.0, -9.8),
                 device: Optional[torch.device] = None):
        self.lib = C.load()
        self.device = device or torch.device("cuda:0")
        self.stream = torch.cuda.Stream(device=self.device)
        L, K, nc = pack_links(links)
        self.E, self.N, self.n_contacts = int(n_envs), len(links), nc
        self.max_substeps = int(max_substeps)
        d = C.mpm_rb_desc()
        d.n_envs, d.n_links, d.n_contacts, d.max_substeps, d.dt = self.E, self.N, nc, self.max_substeps, float(dt)
        d.gravity[:] = [float(g) for g in gravity]
        self.h = ctypes.c_void_p()
        code = self.lib.mpm_rb_create(ctypes.byref(d), L, K, None, ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(self.h))
        C.check(code, "mpm_rb_create")
        self.recorded = None
        self._keep = None
        self.record_token = 0   # changes whenever the library's record is replaced or dropped

    def close(self):
        if self.h:
            self.lib.mpm_rb_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code, where):
        C.check(code, where, self.h, rb=True)

    def _sync_in(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _sync_out(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.E, C.MPM_RB_PARAMS))
        self._chk(self.lib.mpm_rb_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                  "mpm_rb_set_params")
        self.record_token += 1

    def set_state(self, q, qd=None) -> None:
        q = _f32(q, self.device)
        qd = None if qd is None else _f32(qd, self.device)
        self._keep = (q, qd)
        self._sync_in()
        self._chk(self.lib.mpm_rb_set_state(self.h, C.ptr(q), C.ptr(qd)), "mpm_rb_set_state")
        self.recorded = None
        self.record_token += 1

    def get_state(self):
        q = torch.empty(self.E, self.N, device=self.device)
        qd = torch.empty(self.E, self.N, device=self.device)
        self._sync_in()
        self._chk(self.lib.mpm_rb_get_state(self.h, C.ptr(q), C.ptr(qd)), "mpm_rb_get_state")
        self._sync_out()
        return q, qd

    def forward(self, S: int, tau=None, record: bool = False) -> None:
        t = None if tau is None else _f32(tau, self.device)
        if t is not None and tuple(t.shape) != (S, self.E, self.N):
            raise ValueError(f"torques must be [S, E, N] = {(S, self.E, self.N)}, got {tuple(t.shape)}")
        self._keep_tau = t
        self._sync_in()
        self._chk(self.lib.mpm_rb_forward(self.h, int(S), C.ptr(t), C.MPM_FWD_RECORD if record else 0),
                  "mpm_rb_forward")
        self.recorded = int(S) if record else None
        self.record_token += 1

    def backward(self, gq=None, gqd=None, want_tau: bool = True, want_params: bool = True):
        if self.recorded is None:
            raise RuntimeError("backward needs a recorded forward")
        d = self.device
        gq = None if gq is None else _f32(gq, d)
        gqd = None if gqd is None else _f32(gqd, d)
        dq = torch.empty(self.E, self.N, device=d)
        dqd = torch.empty(self.E, self.N, device=d)
        dt = torch.empty(self.recorded, self.E, self.N, device=d) if want_tau else None
        dp = torch.empty(self.E, C.MPM_RB_PARAMS, dtype=torch.float64, device=d) if want_params else None
        self._sync_in()
        self._chk(self.lib.mpm_rb_backward(self.h, C.ptr(gq), C.ptr(gqd), C.ptr(dq), C.ptr(dqd), C.ptr(dt),
                                           C.ptr(dp)), "mpm_rb_backward")
        self._sync_out()
        return dq, dqd, dt, dp

    def sync(self, raise_on_error: bool = True) -> int:
        code = self.lib.mpm_rb_sync(self.h)
        if raise_on_error:
            self._chk(code, "mpm_rb_sync")
        return code

    def env_errors(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.E)()
        self._chk(self.lib.mpm_rb_env_errors(self.h, out), "mpm_rb_env_errors")
        return np.frombuffer(out, dtype=np.int32).copy()

    def memory_bytes(self) -> int:
        return int(self.lib.mpm_rb_memory_bytes(self.h))


class RBRollout(torch.autograd.Function):
    """(q_S, qd_S) = S substeps of the batch from (q0, qd0) with torques tau
    [S, E, N] and per-env parameters params [E, 5] (float64), differentiable
    in all four. If the batch has been used since this call's forward, the
    backward first re-runs the forward from the saved inputs, so calls can be
    chained (one env step after another) in one graph."""

    @staticmethod
    def _run(batch: RbBatch, S: int, q0, qd0, tau, params):
        batch.set_params(params.detach().cpu().numpy())
        batch.set_state(q0.detach(), qd0.detach())
        batch.forward(S, tau.detach(), record=True)

    @staticmethod
    def forward(ctx, batch: RbBatch, S: int, q0, qd0, tau, params):
        RBRollout._run(batch, S, q0, qd0, tau, params)
        q, qd = batch.get_state()
        ctx.batch, ctx.S = batch, S
        ctx.token = batch.record_token
        ctx.save_for_backward(q0, qd0, tau, params)
        return q, qd

    @staticmethod
    def backward(ctx, gq, gqd):
        b = ctx.batch
        q0, qd0, tau, params = ctx.saved_tensors
        if b.record_token != ctx.token:
            RBRollout._run(b, ctx.S, q0, qd0, tau, params)
            ctx.token = b.record_token
        dq, dqd, dt, dp = b.backward(gq, gqd)
        return None, None, dq, dqd, dt, dp.to(device=params.device, dtype=torch.float64)


def rollout(batch: RbBatch, S: int, q0, qd0, tau, params):
    return RBRollout.apply(batch, S, q0, qd0, tau, params)
