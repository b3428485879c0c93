"""Host-side checks of the C interface: the library loads, exports every
function include/mpm.h declares, and rejects bad descriptions before touching
a device."""
import ctypes
import os
import re

import pytest

from paper_2412_12089_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(mpm_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_lists_the_exported_api():
    names = header_functions()
    assert len(names) >= 15
    assert sorted(names) == sorted(C.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = C.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert lib.mpm_version().startswith(b"mpmx")


def _desc(n=32, n_particles=10, dt=1e-4, material=0, wall=3, envs=1, max_substeps=10, K=5, mode=1):
    arr = (C.mpm_env_desc * envs)()
    for d in arr:
        d.n, d.material, d.n_particles, d.dt, d.wall = n, material, n_particles, dt, wall
        d.gravity[:] = [0.0, 0.0, -9.8]
    return C.mpm_batch_desc(envs, arr, max_substeps, K, mode, 0), arr


@pytest.mark.parametrize("kw", [dict(n=30), dict(n=8), dict(dt=0.0), dict(dt=-1.0), dict(material=7),
                                dict(n_particles=-1), dict(wall=15, n=32), dict(K=0), dict(mode=5),
                                dict(max_substeps=-1), dict(envs=0)])
def test_create_rejects_bad_descriptions(kw):
    lib = C.load()
    d, keep = _desc(**kw)
    out = ctypes.c_void_p()
    assert lib.mpm_batch_create(ctypes.byref(d), None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert not out.value


def test_null_arguments_are_rejected():
    lib = C.load()
    out = ctypes.c_void_p()
    assert lib.mpm_batch_create(None, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert lib.mpm_forward(None, 1, 0) == C.MPM_INVALID_ARG
    assert lib.mpm_backward(None, *([None] * 9)) == C.MPM_INVALID_ARG
    assert lib.mpm_sync(None) == C.MPM_INVALID_ARG
    assert lib.mpm_batch_destroy(None) == C.MPM_INVALID_ARG
    assert lib.mpm_last_error(None) == b"null batch"
    assert lib.mpm_memory_bytes(None) == 0


def test_key_width_limit():
    # 2^12 envs of 96^3 nodes need 12 + 20 bits: accepted; 2^13 are rejected before allocation
    lib = C.load()
    d, keep = _desc(n=96, envs=8193, n_particles=0)
    out = ctypes.c_void_p()
    assert lib.mpm_batch_create(ctypes.byref(d), None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
