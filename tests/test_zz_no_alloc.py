"""The allocation-free binning entry point against the batch's own binning
(mpm_sort_keys): bit-exact keys and permutation on two calls in a row, the
second with fewer particles, plus the size check."""
import numpy as np
import pytest
import torch

from conftest import gpu_available
from gpu_util import make_env
from oracle import mpm_oracle as O
from paper_2412_12089_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def boundary_env(n, N, seed):
    # positions exactly on cell boundaries (x n - 1/2 integral), one ulp either side, and repeated keys
    e = make_env(scenes.NEOHOOKEAN, N=N, n=n, seed=seed, lo=0.1, side=0.8)
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(3, n - 4, size=(N // 3, 3))
    xb = ((k + 0.5) / n).astype(np.float32)
    which = rng.integers(0, 3, size=xb.shape)
    xb = np.where(which == 1, np.nextafter(xb, np.float32(0)), xb)
    xb = np.where(which == 2, np.nextafter(xb, np.float32(1)), xb)
    e.x[: len(xb)] = xb
    e.x[len(xb): len(xb) + 5] = e.x[len(xb) + 10]
    return e


def test_sort_keys_noalloc_matches_the_batch_binning():
    from paper_2412_12089_amd import _capi as C
    from paper_2412_12089_amd.batch import Batch
    lib = C.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for n, N, seed in ((96, 300_000, 1), (48, 7_000, 2)):   # the second call is smaller
        e = boundary_env(n, N, seed)
        print(f"[gpu-noalloc] grid {n}^3, {N} particles", flush=True)
        b = Batch([e], max_substeps=1, ckpt_every=1, device=dev)
        b.set_particles_from_specs()
        kb, pb, _, cell_bits = b.sort_keys()
        b.sync()
        b.close()
        x = torch.from_numpy(e.x).to(dev)
        keys = torch.empty(N, dtype=torch.int32, device=dev)
        perm = torch.empty(N, dtype=torch.int32, device=dev)
        rc = lib.mpm_sort_keys_noalloc(C.ptr(x), N, n, C.ptr(keys), C.ptr(perm), stream.cuda_stream)
        assert rc == C.MPM_OK
        torch.cuda.synchronize()
        k = keys.cpu().numpy().view(np.uint32).astype(np.int64)
        p = perm.cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal(k, kb) and np.array_equal(p, pb)
        assert np.array_equal(k, O.cell_keys(e.x, n)) and np.array_equal(p, O.sort_permutation(k))
    # above the scratch size: refused before any device work
    big = C.MPM_SORT_NOALLOC_MAX + 1
    assert lib.mpm_sort_keys_noalloc(C.ptr(x), big, 96, C.ptr(keys), C.ptr(perm), stream.cuda_stream) == C.MPM_INVALID_ARG
