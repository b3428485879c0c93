"""Batched, differentiable MLS-MPM substeps on AMD MI355X (gfx950).

The work is done by libmpmx.so (hand-written HIP kernels behind the C
interface of include/mpm.h); this package marshals torch tensors into it.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "Batch", "MPMRollout", "rollout", "load_library"]


def load_library():
    from . import _capi
    return _capi.load()


def __getattr__(name):
    if name in ("Batch", "MPMRollout", "rollout"):
        from . import batch
        return getattr(batch, name)
    raise AttributeError(name)
