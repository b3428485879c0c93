"""Python face of the C interface: a batch handle and a differentiable rollout.

Argument marshalling only: tensors are handed to libmpmx as device pointers,
torch supplies device memory (through the allocator callbacks) and the
stream, and every step of the substep runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _capi as C
from .scenes import EnvSpec


class TorchAllocator:
    """mpm_allocator backed by torch's caching allocator on one device."""

    def __init__(self, device: torch.device):
        self.device = device
        self.live = {}
        self._alloc = C.ALLOC_FN(self._alloc_impl)
        self._free = C.FREE_FN(self._free_impl)
        self.struct = C.mpm_allocator(self._alloc, self._free, None)

    def _alloc_impl(self, nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free_impl(self, p, ctx):
        self.live.pop(int(p) if p is not None else 0, None)


def _f32(t: torch.Tensor, device) -> torch.Tensor:
    return t.to(device=device, dtype=torch.float32).contiguous()


class Batch:
    """A set of environments simulated together (wraps mpm_batch_*)."""

    def __init__(self, envs: Sequence[EnvSpec], max_substeps: int, ckpt_every: int,
                 mode: str = "batched", device: Optional[torch.device] = None,
                 torch_memory: bool = True, stream: Optional[torch.cuda.Stream] = None):
        self.lib = C.load()
        self.device = torch.device(device or "cuda")
        self.envs = list(envs)
        self.E = len(self.envs)
        self.counts = [e.n_particles for e in self.envs]
        self.N = int(sum(self.counts))
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.max_substeps = int(max_substeps)
        self.ckpt_every = int(ckpt_every)
        self.mode = C.MPM_MODE_PLAIN if mode == "plain" else C.MPM_MODE_BATCHED
        descs = (C.mpm_env_desc * self.E)()
        for d, e in zip(descs, self.envs):
            d.n = e.n
            d.material = e.material
            d.n_particles = e.n_particles
            d.dt = e.dt
            d.gravity[:] = list(e.gravity)
            d.wall = e.wall
        self._descs = descs
        bd = C.mpm_batch_desc(self.E, descs, self.max_substeps, self.ckpt_every, self.mode, 0)
        self.allocator = TorchAllocator(self.device) if torch_memory else None
        self.stream = stream or torch.cuda.current_stream(self.device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            C.check(self.lib.mpm_batch_create(ctypes.byref(bd),
                                              ctypes.byref(self.allocator.struct) if self.allocator else None,
                                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                    "mpm_batch_create")
        self.h = handle
        self.record_token = 0
        for i, e in enumerate(self.envs):
            self.set_material(i, e.material, e.params())
            self._set_all_colliders(i, e)

    def _set_all_colliders(self, env: int, spec) -> None:
        if spec.collider is not None:
            self.set_collider(env, spec.collider)
        for k, c in enumerate(getattr(spec, "more_colliders", ()), start=1):
            self.set_collider(env, c, index=k)

    # -- lifetime
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mpm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, code, where):
        return C.check(code, where, self.h)

    # -- parameters
    def set_material(self, env: int, material: int, params) -> None:
        self.record_token += 1   # the library drops its recorded tape
        p = (ctypes.c_double * 8)(*[float(v) for v in np.asarray(params, dtype=np.float64).reshape(8)])
        self._chk(self.lib.mpm_set_material(self.h, env, material, p), "mpm_set_material")

    def set_box_collider(self, env: int, center, half, velocity, alpha: float, mu_b: float) -> None:
        self.record_token += 1   # the library drops its recorded tape
        f3 = lambda a: (ctypes.c_float * 3)(*[float(x) for x in a])
        self._chk(self.lib.mpm_set_box_collider(self.h, env, f3(center), f3(half), f3(velocity),
                                                float(alpha), float(mu_b)), "mpm_set_box_collider")

    def set_sphere_collider(self, env: int, center, radius: float, velocity, alpha: float, mu_b: float) -> None:
        self.record_token += 1   # the library drops its recorded tape
        f3 = lambda a: (ctypes.c_float * 3)(*[float(x) for x in a])
        self._chk(self.lib.mpm_set_sphere_collider(self.h, env, f3(center), float(radius), f3(velocity),
                                                   float(alpha), float(mu_b)), "mpm_set_sphere_collider")

    def set_rounded_box_collider(self, env: int, center, half, radius: float, velocity, alpha: float,
                                 mu_b: float) -> None:
        self.record_token += 1   # the library drops its recorded tape
        f3 = lambda a: (ctypes.c_float * 3)(*[float(x) for x in a])
        self._chk(self.lib.mpm_set_rounded_box_collider(self.h, env, f3(center), f3(half), float(radius),
                                                        f3(velocity), float(alpha), float(mu_b)),
                  "mpm_set_rounded_box_collider")

    def set_box_rotation(self, env: int, axis, angle: float, omega: float, index: int = 0) -> None:
        self.record_token += 1   # the library drops its recorded tape
        f3 = (ctypes.c_float * 3)(*[float(x) for x in axis])
        self._chk(self.lib.mpm_set_collider_rotation(self.h, env, int(index), f3, float(angle), float(omega)),
                  "mpm_set_collider_rotation")

    def set_collider(self, env: int, c, center=None, angle=None, index: int = 0) -> None:
        """Collider `index` (0 .. MPM_MAX_COLLIDERS - 1) of env: c is a scenes.BoxCollider (a box, a rounded
        box or a ball), optionally with another start center / angle."""
        self.record_token += 1   # the library drops its recorded tape
        cen = c.center if center is None else center
        f3 = lambda a: (ctypes.c_float * 3)(*[float(x) for x in a])
        if getattr(c, "shape", "box") == "sphere":
            shape, radius = C.MPM_COLLIDER_SPHERE, c.half[0]
        elif getattr(c, "rounding", 0.0) > 0.0:
            shape, radius = C.MPM_COLLIDER_ROUNDED_BOX, c.rounding
        else:
            shape, radius = C.MPM_COLLIDER_BOX, 0.0
        self._chk(self.lib.mpm_set_collider(self.h, env, int(index), shape, f3(cen), f3(c.half), float(radius),
                                            f3(c.velocity), float(c.alpha), float(c.mu_b)), "mpm_set_collider")
        if c.alpha > 0.0 and (c.rotates or angle is not None):   # alpha <= 0 removed the collider
            self.set_box_rotation(env, c.axis, c.angle if angle is None else angle, c.omega, index=index)

    def set_collider_motion(self, env: int, vel, omega=None, index: int = 0) -> None:
        """Per-substep velocities [n, 3] and angular speeds [n] (None: the collider's constant one) of
        collider `index`, the actions; vel None or empty clears them."""
        self.record_token += 1   # the library drops its recorded tape
        if vel is None or len(vel) == 0:
            self._chk(self.lib.mpm_set_collider_motion_at(self.h, env, int(index), None, None, 0),
                      "mpm_set_collider_motion_at")
            return
        v = np.ascontiguousarray(np.asarray(vel, dtype=np.float32).reshape(-1, 3))
        buf = v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        ob = None
        if omega is not None:
            o = np.ascontiguousarray(np.asarray(omega, dtype=np.float32).reshape(-1))
            assert o.shape[0] == v.shape[0]
            ob = o.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._chk(self.lib.mpm_set_collider_motion_at(self.h, env, int(index), buf, ob, v.shape[0]),
                  "mpm_set_collider_motion_at")

    def moments(self, x, v, w=None):
        """Per-env weighted moments [E, 20] float64 of caller-order x, v (device)."""
        d = self.device
        x, v = _f32(x, d), _f32(v, d)
        out = torch.empty(self.E, C.MPM_MOMENTS, dtype=torch.float64, device=d)
        self._chk(self.lib.mpm_moments(self.h, C.ptr(x), C.ptr(v), C.ptr(w), C.ptr(out)), "mpm_moments")
        return out

    def moments_vjp(self, x, v, w, g):
        d = self.device
        x, v = _f32(x, d), _f32(v, d)
        g = g.to(d, torch.float64).contiguous()
        gx, gv = torch.empty_like(x), torch.empty_like(v)
        self._chk(self.lib.mpm_moments_vjp(self.h, C.ptr(x), C.ptr(v), C.ptr(w), C.ptr(g), C.ptr(gx), C.ptr(gv)),
                  "mpm_moments_vjp")
        return gx, gv

    def pair_distance(self, x, pairs):
        """[E, 2] float64 (mean distance of each env's particle pairs, pair count); pairs int32 [P, 3] (env, a, b)."""
        d = self.device
        x = _f32(x, d)
        pairs = pairs.to(device=d, dtype=torch.int32).contiguous()
        out = torch.empty(self.E, 2, dtype=torch.float64, device=d)
        self._chk(self.lib.mpm_pair_distance(self.h, C.ptr(x), C.ptr(pairs), int(pairs.shape[0]), C.ptr(out)),
                  "mpm_pair_distance")
        return out

    def pair_distance_vjp(self, x, pairs, out, g):
        d = self.device
        x = _f32(x, d)
        pairs = pairs.to(device=d, dtype=torch.int32).contiguous()
        g = g.to(d, torch.float64).contiguous()
        gx = torch.empty_like(x)
        self._chk(self.lib.mpm_pair_distance_vjp(self.h, C.ptr(x), C.ptr(pairs), int(pairs.shape[0]), C.ptr(out),
                                                 C.ptr(g), C.ptr(gx)), "mpm_pair_distance_vjp")
        return gx

    def collider_grad(self, env: int, n: int, spin: bool = False, index: int = 0):
        """After backward, of collider `index`: (dL/dvel [n, 3], dL/dc0 [3]) in float64, and with spin=True
        also (dL/domega [n], dL/dangle0)."""
        dvel = np.zeros((n, 3), np.float64)
        dc0 = np.zeros(3, np.float64)
        dom = np.zeros(n, np.float64)
        dang = np.zeros(1, np.float64)
        P = ctypes.POINTER(ctypes.c_double)
        self._chk(self.lib.mpm_get_collider_grad_at(self.h, env, int(index), dvel.ctypes.data_as(P),
                                                    dc0.ctypes.data_as(P), dom.ctypes.data_as(P),
                                                    dang.ctypes.data_as(P), n), "mpm_get_collider_grad_at")
        return (dvel, dc0, dom, float(dang[0])) if spin else (dvel, dc0)

    # -- state
    def set_particles(self, x, v, Cm, F, env: int = -1) -> None:
        self.record_token += 1   # the library drops its recorded tape
        d = self.device
        x, v, Cm, F = (_f32(t, d) for t in (x, v, Cm, F))
        n = x.shape[0]
        self._keep = (x, v, Cm, F)   # alive until the copy kernel has run on the stream
        self._chk(self.lib.mpm_set_particles(self.h, env, C.ptr(x), C.ptr(v), C.ptr(Cm), C.ptr(F), n),
                  "mpm_set_particles")

    def set_particles_from_specs(self) -> None:
        cat = lambda k: torch.from_numpy(np.concatenate([getattr(e, k) for e in self.envs], axis=0))
        self.set_particles(cat("x"), cat("v"), cat("C"), cat("F"))

    def get_particles(self, env: int = -1):
        n = self.N if env < 0 else self.counts[env]
        d = self.device
        x = torch.empty(n, 3, device=d)
        v = torch.empty(n, 3, device=d)
        Cm = torch.empty(n, 3, 3, device=d)
        F = torch.empty(n, 3, 3, device=d)
        self._chk(self.lib.mpm_get_particles(self.h, env, C.ptr(x), C.ptr(v), C.ptr(Cm), C.ptr(F)),
                  "mpm_get_particles")
        return x, v, Cm, F

    # -- stepping
    def forward(self, n_substeps: int, record: bool = False) -> None:
        self._chk(self.lib.mpm_forward(self.h, int(n_substeps), C.MPM_FWD_RECORD if record else 0), "mpm_forward")
        self.record_token += 1   # any forward replaces (or drops) the recorded tape

    def forward_envs(self, n_substeps, record: bool = False) -> None:
        arr = (ctypes.c_int32 * self.E)(*[int(k) for k in n_substeps])
        self._chk(self.lib.mpm_forward_envs(self.h, arr, C.MPM_FWD_RECORD if record else 0), "mpm_forward_envs")
        self.record_token += 1

    def configure_env(self, env: int, spec: EnvSpec) -> None:
        """Re-describe slot `env` (within its capacity) and set its material and particles."""
        self.record_token += 1   # the library drops its recorded tape
        d = C.mpm_env_desc()
        d.n, d.material, d.n_particles, d.dt, d.wall = spec.n, spec.material, spec.n_particles, spec.dt, spec.wall
        d.gravity[:] = list(spec.gravity)
        self._chk(self.lib.mpm_configure_env(self.h, env, ctypes.byref(d)), "mpm_configure_env")
        self.counts[env] = spec.n_particles
        self.N = int(sum(self.counts))
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.envs[env] = spec
        self.set_material(env, spec.material, spec.params())
        self._set_all_colliders(env, spec)

    def backward(self, gx=None, gv=None, gC=None, gF=None, want_params: bool = True):
        d = self.device
        cv = lambda t: None if t is None else _f32(t, d)
        gx, gv, gC, gF = cv(gx), cv(gv), cv(gC), cv(gF)
        self._keep_cot = (gx, gv, gC, gF)
        dx = torch.empty(self.N, 3, device=d)
        dv = torch.empty(self.N, 3, device=d)
        dC = torch.empty(self.N, 3, 3, device=d)
        dF = torch.empty(self.N, 3, 3, device=d)
        dp = torch.empty(self.E, 8, dtype=torch.float64, device=d) if want_params else None
        self._chk(self.lib.mpm_backward(self.h, C.ptr(gx), C.ptr(gv), C.ptr(gC), C.ptr(gF), C.ptr(dx), C.ptr(dv),
                                        C.ptr(dC), C.ptr(dF), C.ptr(dp)), "mpm_backward")
        return dx, dv, dC, dF, dp

    def sort_keys(self):
        """(keys uint32 as int64, perm int64, ids int64, cell_bits) of the current state."""
        keys = torch.empty(self.N, dtype=torch.int32, device=self.device)
        perm = torch.empty(self.N, dtype=torch.int32, device=self.device)
        ids = torch.empty(self.N, dtype=torch.int32, device=self.device)
        cb = ctypes.c_int32()
        self._chk(self.lib.mpm_sort_keys(self.h, C.ptr(keys), C.ptr(perm), C.ptr(ids), ctypes.byref(cb)),
                  "mpm_sort_keys")
        u = lambda t: t.cpu().numpy().view(np.uint32).astype(np.int64)
        return u(keys), u(perm), ids.cpu().numpy().astype(np.int64), int(cb.value)

    def sync(self, raise_on_error: bool = True) -> int:
        code = self.lib.mpm_sync(self.h)
        if raise_on_error:
            self._chk(code, "mpm_sync")
        return code

    def env_errors(self) -> np.ndarray:
        out = (ctypes.c_int32 * self.E)()
        self._chk(self.lib.mpm_env_errors(self.h, out), "mpm_env_errors")
        return np.frombuffer(out, dtype=np.int32).copy()

    def autotune(self, budget_ms: int = 200) -> None:
        self._chk(self.lib.mpm_autotune(self.h, int(budget_ms)), "mpm_autotune")

    def set_option(self, option: int, value: int) -> None:
        self._chk(self.lib.mpm_set_option(self.h, int(option), int(value)), "mpm_set_option")

    def get_option(self, option: int) -> int:
        v = ctypes.c_int32()
        self._chk(self.lib.mpm_get_option(self.h, int(option), ctypes.byref(v)), "mpm_get_option")
        return int(v.value)

    def memory_bytes(self) -> int:
        return int(self.lib.mpm_memory_bytes(self.h))

    def set_timing(self, on: bool) -> None:
        self._chk(self.lib.mpm_set_timing(self.h, 1 if on else 0), "mpm_set_timing")

    def kernel_time(self, name: str):
        ms = ctypes.c_double()
        n = self.lib.mpm_kernel_time(self.h, C.KERNEL_CLASSES.index(name), ctypes.byref(ms))
        return ms.value, int(n)


def _slots(spec) -> list:
    """The env's colliders by slot (slot 0: `collider`, then `more_colliders`; None where a slot is empty)."""
    return [spec.collider] + list(getattr(spec, "more_colliders", ()))


class MPMRollout(torch.autograd.Function):
    """s_S = f^S(s_0; params, actions, centers, spins) through the library,
    differentiable in s_0, params, actions, centers and spins.

    params: [E, 8] float64 (E, nu, rho, Vp, sigma_y, K, gamma, 0) per env.
    actions: None, [E, S, 3] per-substep velocities of each env's first
    collider, or [E, K, S, 3] of its colliders in slots 0 .. K-1; spins: None,
    [E, S] or [E, K, S] per-substep angular speeds about each collider's axis
    (needs actions; default: the collider's constant angular speed); centers:
    None, [E, 3] or [E, K, 3] the colliders' centers at the first substep
    (default: the centers the envs were created with). Rows of empty slots are
    ignored and get zero gradients. If the batch has been re-used since this
    call's forward, the backward first re-runs the forward from the saved
    inputs (frame-level checkpoint), so calls can be chained.
    """

    @staticmethod
    def _per_slot(t, dims):
        """[E, K, ...] view of an input given per slot or for slot 0 alone."""
        if t is None:
            return None
        return t if t.dim() == dims + 1 else t.unsqueeze(1)

    @staticmethod
    def _setup(batch: Batch, n_substeps: int, x, v, Cm, F, params, actions, centers, spins):
        prm = params.detach().to("cpu", torch.float64).numpy()
        for i, e in enumerate(batch.envs):
            batch.set_material(i, e.material, prm[i])
        cen = MPMRollout._per_slot(centers, 2)
        if cen is not None:
            cen = cen.detach().to("cpu", torch.float64).numpy()
            for i, e in enumerate(batch.envs):
                for k, c in enumerate(_slots(e)[:cen.shape[1]]):
                    if c is not None:
                        batch.set_collider(i, c, center=cen[i, k], index=k)
        act = MPMRollout._per_slot(actions, 3)
        if act is not None:
            act = act.detach().to("cpu", torch.float32).numpy()
            spn = MPMRollout._per_slot(spins, 2)
            spn = None if spn is None else spn.detach().to("cpu", torch.float32).numpy()
            for i, e in enumerate(batch.envs):
                for k, c in enumerate(_slots(e)[:act.shape[1]]):
                    if c is not None:
                        batch.set_collider_motion(i, act[i, k, :n_substeps],
                                                  None if spn is None else spn[i, k, :n_substeps], index=k)
        batch.set_particles(x, v, Cm, F)
        batch.forward(n_substeps, record=True)

    @staticmethod
    def forward(ctx, batch: Batch, n_substeps: int, x, v, Cm, F, params, actions=None, centers=None, spins=None):
        if spins is not None and actions is None:
            raise ValueError("spins need actions (a prescribed motion)")
        MPMRollout._setup(batch, n_substeps, x, v, Cm, F, params, actions, centers, spins)
        ctx.batch = batch
        ctx.n_substeps = n_substeps
        ctx.token = batch.record_token
        ctx.flags = (actions is not None, centers is not None, spins is not None)
        empty = torch.empty(0)
        ctx.save_for_backward(x, v, Cm, F, params, actions if actions is not None else empty,
                              centers if centers is not None else empty, spins if spins is not None else empty)
        return batch.get_particles()

    @staticmethod
    def backward(ctx, gx, gv, gC, gF):
        b = ctx.batch
        x, v, Cm, F, params, actions, centers, spins = ctx.saved_tensors
        actions = actions if ctx.flags[0] else None
        centers = centers if ctx.flags[1] else None
        spins = spins if ctx.flags[2] else None
        if b.record_token != ctx.token:
            MPMRollout._setup(b, ctx.n_substeps, x, v, Cm, F, params, actions, centers, spins)
            ctx.token = b.record_token
        dx, dv, dC, dF, dp = b.backward(gx, gv, gC, gF)
        da = dcen = dsp = None
        if actions is not None:
            act = MPMRollout._per_slot(actions, 3)
            K, S = act.shape[1], act.shape[2]
            da = torch.zeros(b.E, K, S, 3, dtype=torch.float64)
            dcen = torch.zeros(b.E, K, 3, dtype=torch.float64)
            dsp = torch.zeros(b.E, K, S, dtype=torch.float64)
            for i, e in enumerate(b.envs):
                for k, c in enumerate(_slots(e)[:K]):
                    if c is not None:
                        dvel, dc0, dom, _ = b.collider_grad(i, ctx.n_substeps, spin=True, index=k)
                        da[i, k, :ctx.n_substeps] = torch.from_numpy(dvel)
                        dcen[i, k] = torch.from_numpy(dc0)
                        dsp[i, k, :ctx.n_substeps] = torch.from_numpy(dom)
            da = da.reshape(actions.shape).to(actions.device, actions.dtype)
        if centers is None:
            dcen = None
        else:
            if dcen is None:   # a fixed-velocity collider: the start center matters, its gradient is not computed
                raise ValueError("gradients w.r.t. centers need actions (a prescribed motion)")
            dcen = dcen[:, :MPMRollout._per_slot(centers, 2).shape[1]].reshape(centers.shape)
            dcen = dcen.to(centers.device, centers.dtype)
        if spins is None:
            dsp = None
        else:
            sp = MPMRollout._per_slot(spins, 2)
            dsp = dsp[:, :sp.shape[1], :sp.shape[2]].reshape(spins.shape).to(spins.device, spins.dtype)
        return None, None, dx, dv, dC, dF, dp.to(params.device, params.dtype), da, dcen, dsp


def rollout(batch: Batch, n_substeps: int, x, v, Cm, F, params, actions=None, centers=None, spins=None):
    return MPMRollout.apply(batch, n_substeps, x, v, Cm, F, params, actions, centers, spins)
