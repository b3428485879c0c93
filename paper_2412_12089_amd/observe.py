"""Observation / reward statistics of the manipulation tasks on the device.

Per-env weighted moments of particle positions and velocities (libmpmx
mpm_moments, FP64 accumulation) behind a torch.autograd.Function whose
backward is the library's mpm_moments_vjp; the task statistics (centre of
mass of a subsampled particle set, height variance, mean velocity) are a few
divisions of those moments.
"""
from __future__ import annotations

import torch

from . import _capi as C


class Moments(torch.autograd.Function):
    """[E, 20] float64 moments of caller-order x, v [rows, 3] (float32, device)."""

    @staticmethod
    def forward(ctx, batch, x, v, w=None):
        x, v = x.contiguous(), v.contiguous()
        w = None if w is None else w.contiguous().float()
        out = batch.moments(x, v, w)
        ctx.batch = batch
        ctx.save_for_backward(x, v, w if w is not None else torch.empty(0))
        ctx.has_w = w is not None
        return out

    @staticmethod
    def backward(ctx, g):
        x, v, w = ctx.saved_tensors
        gx, gv = ctx.batch.moments_vjp(x, v, w if ctx.has_w else None, g.contiguous().double())
        return None, gx, gv, None


def moments(batch, x, v, w=None):
    return Moments.apply(batch, x, v, w)


def center_of_mass(m):
    return m[:, 1:4] / m[:, :1]


def height_variance(m):
    return m[:, 6] / m[:, 0] - (m[:, 3] / m[:, 0]) ** 2


def mean_velocity(m):
    return m[:, 10:13] / m[:, :1]


def subsample_weights(batch, stride: int):
    """0/1 weights that keep every stride-th particle of each env (caller order)."""
    w = torch.zeros(batch.N, dtype=torch.float32, device=batch.device)
    off = 0
    for n in batch.counts:
        w[off:off + n:stride] = 1.0
        off += n
    return w
