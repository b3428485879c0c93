"""Python binding of the FEM batch (include/mpm_fem.h): argument marshalling only.

`FemBatch` owns a library handle and passes torch CUDA tensors by address;
every step runs in the library's HIP kernels. `FEMRollout` makes a recorded
forward and its adjoint an autograd Function, differentiable in the initial
state, the activations and the per-env parameters; calls on one batch can be
chained (a backward whose record was replaced re-runs its forward first).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _capi as C


def _f32(t, device) -> torch.Tensor:
    return torch.as_tensor(t, dtype=torch.float32, device=device).contiguous()


class FemBatch:
    """E soft bodies sharing one tetrahedral mesh (tets [T, 4])."""

    def __init__(self, tets, n_envs: int, n_nodes: int, max_substeps: int, dt: float,
                 gravity=(0.0, 0.0, -9.8), device: Optional[torch.device] = None):
        self.lib = C.load()
        self.device = device or torch.device("cuda:0")
        self.stream = torch.cuda.Stream(device=self.device)
        tets = np.ascontiguousarray(np.asarray(tets, dtype=np.int32))
        self.E, self.n, self.T = int(n_envs), int(n_nodes), int(tets.shape[0])
        self.max_substeps = int(max_substeps)
        d = C.mpm_fem_desc()
        d.n_envs, d.n_nodes, d.n_tets, d.max_substeps, d.dt = self.E, self.n, self.T, self.max_substeps, float(dt)
        d.gravity[:] = [float(g) for g in gravity]
        self.h = ctypes.c_void_p()
        code = self.lib.mpm_fem_create(ctypes.byref(d), tets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.h))
        C.check(code, "mpm_fem_create")
        self.recorded = None
        self._keep = None
        self.record_token = 0   # changes whenever the library's record is replaced or dropped

    def close(self):
        if self.h:
            self.lib.mpm_fem_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code, where):
        C.check(code, where, self.h, fem=True)

    def _sync_in(self):
        # the library's stream waits for torch's current stream (inputs written there)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _sync_out(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_rest(self, X) -> None:
        X = _f32(X, self.device)
        self._sync_in()
        self._chk(self.lib.mpm_fem_set_rest(self.h, C.ptr(X)), "mpm_fem_set_rest")
        self.recorded = None
        self.record_token += 1

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(self.E, C.MPM_FEM_PARAMS))
        self._chk(self.lib.mpm_fem_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                  "mpm_fem_set_params")
        self.record_token += 1

    def set_state(self, x, v=None) -> None:
        x = _f32(x, self.device)
        v = None if v is None else _f32(v, self.device)
        self._keep = (x, v)
        self._sync_in()
        self._chk(self.lib.mpm_fem_set_state(self.h, C.ptr(x), C.ptr(v)), "mpm_fem_set_state")
        self.recorded = None
        self.record_token += 1

    def get_state(self):
        x = torch.empty(self.E, self.n, 3, device=self.device)
        v = torch.empty(self.E, self.n, 3, device=self.device)
        self._sync_in()
        self._chk(self.lib.mpm_fem_get_state(self.h, C.ptr(x), C.ptr(v)), "mpm_fem_get_state")
        self._sync_out()
        return x, v

    def forward(self, S: int, act=None, record: bool = False) -> None:
        a = None if act is None else _f32(act, self.device)
        if a is not None and tuple(a.shape) != (S, self.E, self.T):
            raise ValueError(f"activations must be [S, E, T] = {(S, self.E, self.T)}, got {tuple(a.shape)}")
        self._keep_act = a
        self._sync_in()
        self._chk(self.lib.mpm_fem_forward(self.h, int(S), C.ptr(a), C.MPM_FWD_RECORD if record else 0),
                  "mpm_fem_forward")
        self.recorded = int(S) if record else None
        self.record_token += 1

    def backward(self, gx=None, gv=None, want_act: bool = True, want_params: bool = True):
        if self.recorded is None:
            raise RuntimeError("backward needs a recorded forward")
        d = self.device
        gx = None if gx is None else _f32(gx, d)
        gv = None if gv is None else _f32(gv, d)
        dx = torch.empty(self.E, self.n, 3, device=d)
        dv = torch.empty(self.E, self.n, 3, device=d)
        da = torch.empty(self.recorded, self.E, self.T, device=d) if want_act else None
        dp = torch.empty(self.E, C.MPM_FEM_PARAMS, dtype=torch.float64, device=d) if want_params else None
        self._sync_in()
        self._chk(self.lib.mpm_fem_backward(self.h, C.ptr(gx), C.ptr(gv), C.ptr(dx), C.ptr(dv), C.ptr(da),
                                            C.ptr(dp)), "mpm_fem_backward")
        self._sync_out()
        return dx, dv, da, dp

    def sync(self, raise_on_error: bool = True) -> int:
        code = self.lib.mpm_fem_sync(self.h)
        if raise_on_error:
            self._chk(code, "mpm_fem_sync")
        return code

    def env_errors(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.E)()
        self._chk(self.lib.mpm_fem_env_errors(self.h, out), "mpm_fem_env_errors")
        return np.frombuffer(out, dtype=np.int32).copy()

    def memory_bytes(self) -> int:
        return int(self.lib.mpm_fem_memory_bytes(self.h))


class FEMRollout(torch.autograd.Function):
    """(x_S, v_S) = S substeps of the batch from (x0, v0) with activations act
    [S, E, T] and per-env parameters params [E, 8] (float64), differentiable
    in all four. The batch's rest shape is fixed. If the batch has been used
    since this call's forward, the backward first re-runs the forward from
    the saved inputs, so calls can be chained in one graph."""

    @staticmethod
    def _run(batch: FemBatch, S: int, x0, v0, act, params):
        batch.set_params(params.detach().cpu().numpy())
        batch.set_state(x0.detach(), v0.detach())
        batch.forward(S, act.detach(), record=True)

    @staticmethod
    def forward(ctx, batch: FemBatch, S: int, x0, v0, act, params):
        FEMRollout._run(batch, S, x0, v0, act, params)
        x, v = batch.get_state()
        ctx.batch, ctx.S = batch, S
        ctx.token = batch.record_token
        ctx.save_for_backward(x0, v0, act, params)
        return x, v

    @staticmethod
    def backward(ctx, gx, gv):
        b = ctx.batch
        x0, v0, act, params = ctx.saved_tensors
        if b.record_token != ctx.token:
            FEMRollout._run(b, ctx.S, x0, v0, act, params)
            ctx.token = b.record_token
        dx, dv, da, dp = b.backward(gx, gv)
        return None, None, dx, dv, da, dp.to(device=params.device, dtype=torch.float64)


def rollout(batch: FemBatch, S: int, x0, v0, act, params):
    return FEMRollout.apply(batch, S, x0, v0, act, params)
