"""Host-side checks of the C interface: the library loads, exports every
function include/*.h declares, and rejects bad descriptions before touching
a device."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_2412_12089_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
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
    f3 = (ctypes.c_float * 3)(0.5, 0.5, 0.5)
    assert lib.mpm_set_collider(None, 0, 1, C.MPM_COLLIDER_SPHERE, f3, f3, 0.1, f3, 10.0, 0.1) == C.MPM_INVALID_ARG
    assert lib.mpm_set_collider_rotation(None, 0, 1, f3, 0.0, 1.0) == C.MPM_INVALID_ARG
    assert lib.mpm_set_collider_motion_at(None, 0, 1, None, None, 0) == C.MPM_INVALID_ARG
    assert lib.mpm_get_collider_grad_at(None, 0, 1, None, None, None, None, 0) == C.MPM_INVALID_ARG


def test_key_width_limit():
    # 2^12 envs of 96^3 nodes need 12 + 20 bits: accepted; 2^13 are rejected before allocation
    lib = C.load()
    d, keep = _desc(n=96, envs=8193, n_particles=0)
    out = ctypes.c_void_p()
    assert lib.mpm_batch_create(ctypes.byref(d), None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG


def _fem_desc(E=2, n=12, T=12, S=4, dt=1e-4):
    d = C.mpm_fem_desc()
    d.n_envs, d.n_nodes, d.n_tets, d.max_substeps, d.dt = E, n, T, S, dt
    d.gravity[:] = [0.0, 0.0, -9.8]
    return d


def _fem_tets(T=12, n=12):
    rng = np.random.default_rng(0)
    return np.stack([rng.choice(n, 4, replace=False) for _ in range(T)]).astype(np.int32)


@pytest.mark.parametrize("kw", [dict(E=0), dict(n=3), dict(n=513), dict(T=0), dict(T=1025), dict(S=-1),
                                dict(dt=0.0), dict(dt=float("nan"))])
def test_fem_create_rejects_bad_descriptions(kw):
    lib = C.load()
    d = _fem_desc(**kw)
    tets = _fem_tets(min(max(d.n_tets, 1), 1024), max(d.n_nodes, 4))
    out = ctypes.c_void_p()
    ptr = tets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.mpm_fem_create(ctypes.byref(d), ptr, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert not out.value


@pytest.mark.parametrize("bad", ["range", "negative", "repeat", "orphan"])
def test_fem_create_rejects_bad_topology(bad):
    lib = C.load()
    d = _fem_desc()
    tets = _fem_tets()
    if bad == "orphan":   # elements over nodes 0..10 only: node 11 has no element
        tets = _fem_tets(12, 11)
    else:
        tets[5] = {"range": [0, 1, 2, 12], "negative": [0, -1, 2, 3], "repeat": [4, 5, 4, 6]}[bad]
    out = ctypes.c_void_p()
    ptr = tets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.mpm_fem_create(ctypes.byref(d), ptr, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert not out.value


def test_fem_null_arguments_are_rejected():
    lib = C.load()
    out = ctypes.c_void_p()
    assert lib.mpm_fem_create(None, None, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    for fn, nargs in (("mpm_fem_destroy", 0), ("mpm_fem_set_rest", 1), ("mpm_fem_set_params", 1),
                      ("mpm_fem_set_state", 2), ("mpm_fem_get_state", 2), ("mpm_fem_backward", 6),
                      ("mpm_fem_sync", 0), ("mpm_fem_env_errors", 1)):
        assert getattr(lib, fn)(None, *([None] * nargs)) == C.MPM_INVALID_ARG, fn
    assert lib.mpm_fem_forward(None, 1, None, 0) == C.MPM_INVALID_ARG
    assert lib.mpm_fem_memory_bytes(None) == 0
    assert lib.mpm_fem_last_error(None) == b"null FEM batch"


def _rb(N=4, C_=2, E=2, S=4, dt=1e-3):
    from paper_2412_12089_amd import rb_scenes as RS
    from paper_2412_12089_amd.rb import pack_links
    links = RS.random_tree(3, N, n_contacts=C_)
    d = C.mpm_rb_desc()
    L, K, nc = pack_links(links)
    d.n_envs, d.n_links, d.n_contacts, d.max_substeps, d.dt = E, N, nc, S, dt
    d.gravity[:] = [0.0, 0.0, -9.8]
    return d, L, K


@pytest.mark.parametrize("kw", [dict(E=0), dict(N=65), dict(S=-1), dict(dt=0.0), dict(dt=float("nan"))])
def test_rb_create_rejects_bad_descriptions(kw):
    lib = C.load()
    N = kw.pop("N", 4)
    d, L, K = _rb(N=min(N, 64), **kw)
    d.n_links = N
    if N > 64:
        L = (C.mpm_rb_link * N)(*L, *[L[0]] * (N - 64))
    out = ctypes.c_void_p()
    assert lib.mpm_rb_create(ctypes.byref(d), L, K, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert not out.value


@pytest.mark.parametrize("bad", ["root", "order", "axis", "rotation", "reflection", "mass", "contact_link",
                                 "radius", "contacts", "joint"])
def test_rb_create_rejects_bad_links(bad):
    lib = C.load()
    d, L, K = _rb()
    if bad == "root":
        L[0].parent = 1
    elif bad == "order":
        L[2].parent = 3
    elif bad == "axis":
        L[1].axis[:] = [1.0, 1.0, 0.0]
    elif bad == "rotation":
        L[1].joint_rot[0] *= 1.01
    elif bad == "reflection":
        L[1].joint_rot[:] = [1, 0, 0, 0, 1, 0, 0, 0, -1]
    elif bad == "mass":
        L[3].mass = -0.1
    elif bad == "contact_link":
        K[0].link = 4
    elif bad == "radius":
        K[1].radius = -0.01
    elif bad == "contacts":
        d.n_contacts = 257
    elif bad == "joint":
        L[2].joint = 2
    out = ctypes.c_void_p()
    assert lib.mpm_rb_create(ctypes.byref(d), L, K, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    assert not out.value


def test_rb_null_arguments_are_rejected():
    lib = C.load()
    out = ctypes.c_void_p()
    assert lib.mpm_rb_create(None, None, None, None, None, ctypes.byref(out)) == C.MPM_INVALID_ARG
    for fn, nargs in (("mpm_rb_destroy", 0), ("mpm_rb_set_params", 1), ("mpm_rb_set_state", 2),
                      ("mpm_rb_get_state", 2), ("mpm_rb_backward", 6), ("mpm_rb_sync", 0),
                      ("mpm_rb_env_errors", 1)):
        assert getattr(lib, fn)(None, *([None] * nargs)) == C.MPM_INVALID_ARG, fn
    assert lib.mpm_rb_forward(None, 1, None, 0) == C.MPM_INVALID_ARG
    assert lib.mpm_rb_memory_bytes(None) == 0
    assert lib.mpm_rb_last_error(None) == b"null rigid-body batch"
