"""Observation / reward statistics of the manipulation tasks on the device.

Per-env weighted moments of particle positions and velocities (libmpmx
mpm_moments, FP64 accumulation) behind a torch.autograd.Function whose
backward is the library's mpm_moments_vjp; the task statistics (centre of
mass of a subsampled particle set, height variance, mean velocity) are a few
divisions of those moments. The flip reward of the HandFlip task (paper
Appendix E) is the per-env mean distance of mirrored particle pairs
(mpm_pair_distance and its VJP) and its normalized improvement over the
initial value.
"""
from __future__ import annotations

import numpy as np
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


class PairDistance(torch.autograd.Function):
    """[E] float64: per-env mean distance of the pairs (env, a, b) of caller-order x [rows, 3]."""

    @staticmethod
    def forward(ctx, batch, x, pairs):
        x = x.contiguous()
        out = batch.pair_distance(x, pairs)
        ctx.batch = batch
        ctx.save_for_backward(x, pairs, out)
        return out[:, 0].clone()

    @staticmethod
    def backward(ctx, g):
        x, pairs, out = ctx.saved_tensors
        return None, ctx.batch.pair_distance_vjp(x, pairs, out, g.contiguous()), None


def flip_distance(batch, x, pairs):
    return PairDistance.apply(batch, x, pairs)


def normalized_improvement(r, r0):
    """NI{r} = clamp((r0 - r) / r0, -1, 1), the HandFlip reward of the flip distance r."""
    return torch.clamp((r0 - r) / r0, -1.0, 1.0)


def mirror_pairs(counts, x0, axis: int = 2, plane=None):
    """Pairs (env, lower, upper) of each env's particles mirrored across the plane
    x[axis] = plane (default: the env's mean along the axis). counts: particles per
    env (the batch's counts); x0: caller-order positions [rows, 3] (host or
    device). Each particle below the plane is matched to the upper-half particle
    nearest to its mirror image (k-d tree)."""
    from scipy.spatial import cKDTree
    x0 = np.asarray(x0.detach().cpu().numpy() if torch.is_tensor(x0) else x0, dtype=np.float64)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    out = []
    for e, (lo, hi) in enumerate(zip(offsets[:-1], offsets[1:])):
        xe = x0[lo:hi]
        if len(xe) == 0:
            continue
        c = float(xe[:, axis].mean()) if plane is None else float(plane)
        low = np.nonzero(xe[:, axis] < c)[0]
        up = np.nonzero(xe[:, axis] >= c)[0]
        if len(low) == 0 or len(up) == 0:
            continue
        img = xe[low].copy()
        img[:, axis] = 2.0 * c - img[:, axis]
        _, j = cKDTree(xe[up]).query(img)
        out.append(np.stack([np.full(len(low), e), low, up[j]], axis=1))
    p = np.concatenate(out, axis=0) if out else np.zeros((0, 3), np.int64)
    return torch.from_numpy(p.astype(np.int32))
