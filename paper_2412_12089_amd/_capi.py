"""ctypes declarations of the C interface in include/mpm.h, include/mpm_fem.h and
include/mpm_rb.h (argument marshalling only).

Every function here has the name and argument order of its C counterpart.
Device arrays are passed as torch CUDA tensors (or None for a NULL pointer);
the library does all the work on the device. Loading fails loudly when the
built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpmx.so")

MPM_OK = 0
MPM_INVALID_ARG = 1
MPM_OUT_OF_MEMORY = 2
MPM_DEVICE_ERROR = 3
MPM_NONFINITE = 4
MPM_OUT_OF_DOMAIN = 5
MPM_BAD_STATE = 6
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE_ERROR", 4: "NONFINITE",
                5: "OUT_OF_DOMAIN", 6: "BAD_STATE"}

MPM_MODE_PLAIN = 0
MPM_MODE_BATCHED = 1
MPM_FWD_RECORD = 1

KERNEL_CLASSES = ("p2g", "grid", "g2p", "sort", "g2p_adj", "grid_adj", "p2g_adj", "g2p2g", "adj_pair")

# every symbol include/*.h declares
EXPORTED = (
    "mpm_batch_create", "mpm_batch_destroy", "mpm_set_particles", "mpm_get_particles", "mpm_set_material",
    "mpm_set_box_collider", "mpm_forward", "mpm_backward", "mpm_autotune", "mpm_sync", "mpm_env_errors",
    "mpm_memory_bytes", "mpm_kernel_time", "mpm_set_timing", "mpm_last_error", "mpm_version", "mpm_sort_keys",
    "mpm_set_option", "mpm_get_option", "mpm_forward_envs", "mpm_configure_env", "mpm_set_collider_motion",
    "mpm_get_collider_grad", "mpm_moments", "mpm_moments_vjp",
    "mpm_server_create", "mpm_server_destroy", "mpm_server_submit", "mpm_server_step", "mpm_server_poll",
    "mpm_server_cancel", "mpm_server_now", "mpm_server_idle", "mpm_server_stats_get", "mpm_server_last_error",
    "mpm_sort_keys_noalloc", "mpm_pair_distance", "mpm_pair_distance_vjp", "mpm_set_box_rotation",
    "mpm_set_sphere_collider", "mpm_set_rounded_box_collider", "mpm_set_collider", "mpm_set_collider_rotation",
    "mpm_set_collider_motion_at", "mpm_get_collider_grad_at",
    "mpm_fem_create", "mpm_fem_destroy", "mpm_fem_set_rest", "mpm_fem_set_params", "mpm_fem_set_state",
    "mpm_fem_get_state", "mpm_fem_forward", "mpm_fem_backward", "mpm_fem_sync", "mpm_fem_env_errors",
    "mpm_fem_last_error", "mpm_fem_memory_bytes",
    "mpm_rb_create", "mpm_rb_destroy", "mpm_rb_set_params", "mpm_rb_set_state", "mpm_rb_get_state",
    "mpm_rb_forward", "mpm_rb_backward", "mpm_rb_sync", "mpm_rb_env_errors", "mpm_rb_last_error",
    "mpm_rb_memory_bytes",
)
MPM_FEM_MAX_NODES = 512
MPM_FEM_MAX_TETS = 1024
MPM_FEM_PARAMS = 8
MPM_RB_MAX_LINKS = 64
MPM_RB_MAX_CONTACTS = 256
MPM_RB_PARAMS = 5
MPM_RB_REVOLUTE = 0
MPM_RB_PRISMATIC = 1
MPM_MAX_COLLIDERS = 4
MPM_COLLIDER_BOX, MPM_COLLIDER_SPHERE, MPM_COLLIDER_ROUNDED_BOX = 1, 2, 3
MPM_SORT_NOALLOC_MAX = 1 << 20
MPM_MOMENTS = 20
(OPT_GRAPHS, OPT_P2G, OPT_G2P, OPT_G2P_ADJ, OPT_P2G_ADJ, OPT_MIN_RUN, OPT_GRID_CAP, OPT_MAX_RUN, OPT_BOX, OPT_SPECIALIZE,
 OPT_FUSE, OPT_FUSE_ADJ, OPT_XCD, OPT_GRID_LIST) = range(1, 15)


class mpm_env_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("material", ctypes.c_int32), ("n_particles", ctypes.c_int64),
                ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3), ("wall", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class mpm_batch_desc(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("envs", ctypes.POINTER(mpm_env_desc)),
                ("max_substeps", ctypes.c_int32), ("ckpt_every", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


MPM_SERVER_DRY = 1
(MPM_REQ_QUEUED, MPM_REQ_RUNNING, MPM_REQ_DONE, MPM_REQ_ERROR, MPM_REQ_CANCELLED, MPM_REQ_REJECTED,
 MPM_REQ_UNKNOWN) = range(7)
REQ_STATE_NAMES = ("queued", "running", "ok", "error", "cancelled", "rejected", "unknown")


class mpm_server_desc(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("n_cap", ctypes.c_int32), ("n_cap_particles", ctypes.c_int64),
                ("chunk", ctypes.c_int32), ("flags", ctypes.c_int32), ("budget_bytes", ctypes.c_int64)]


class mpm_collider(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("center", ctypes.c_float * 3), ("half", ctypes.c_float * 3),
                ("radius", ctypes.c_float), ("vel", ctypes.c_float * 3), ("alpha", ctypes.c_float),
                ("mu_b", ctypes.c_float)]


class mpm_request(ctypes.Structure):
    _fields_ = [("env", mpm_env_desc), ("params", ctypes.c_double * 8), ("has_collider", ctypes.c_int32),
                ("substeps", ctypes.c_int32), ("c_center", ctypes.c_float * 3), ("c_half", ctypes.c_float * 3),
                ("c_vel", ctypes.c_float * 3), ("c_alpha", ctypes.c_float), ("c_mu", ctypes.c_float),
                ("backward", ctypes.c_int32), ("c_round", ctypes.c_float), ("arrival", ctypes.c_double)] + \
               [(k, ctypes.c_void_p) for k in ("x", "v", "C", "F", "gx", "gv", "gC", "gF", "out_x", "out_v", "out_C",
                                                "out_F", "dx0", "dv0", "dC0", "dF0")] + \
               [("n_more", ctypes.c_int32), ("more", mpm_collider * 3)]


class mpm_request_status(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("error_bits", ctypes.c_int32), ("arrival", ctypes.c_double),
                ("admitted", ctypes.c_double), ("finished", ctypes.c_double), ("dparams", ctypes.c_double * 8)]


class mpm_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "done", "errors", "cancelled", "rejected", "queued",
                                              "running", "particle_substeps", "steps")] + \
               [("max_running", ctypes.c_int32), ("reserved", ctypes.c_int32), ("bytes_in_use", ctypes.c_int64)] + \
               [(k, ctypes.c_double) for k in ("p50_ms", "p99_ms", "first_arrival", "last_finish")]


class mpm_fem_desc(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_nodes", ctypes.c_int32), ("n_tets", ctypes.c_int32),
                ("max_substeps", ctypes.c_int32), ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("reserved", ctypes.c_int32 * 4)]


class mpm_rb_desc(ctypes.Structure):
    _fields_ = [("n_envs", ctypes.c_int32), ("n_links", ctypes.c_int32), ("n_contacts", ctypes.c_int32),
                ("max_substeps", ctypes.c_int32), ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("reserved", ctypes.c_int32 * 4)]


class mpm_rb_link(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("joint_rot", ctypes.c_float * 9), ("joint_pos", ctypes.c_float * 3),
                ("axis", ctypes.c_float * 3), ("mass", ctypes.c_float), ("com", ctypes.c_float * 3),
                ("inertia", ctypes.c_float * 6), ("joint", ctypes.c_int32)]


class mpm_rb_contact(ctypes.Structure):
    _fields_ = [("link", ctypes.c_int32), ("centre", ctypes.c_float * 3), ("radius", ctypes.c_float)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mpm_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmpmx.so and declare its prototypes (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() (hipcc for gfx950)")
    lib = ctypes.CDLL(path)
    P, I32, I64, VP = ctypes.POINTER, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    F3 = P(ctypes.c_float)
    D8 = P(ctypes.c_double)
    sig = {
        "mpm_batch_create": (I32, [P(mpm_batch_desc), P(mpm_allocator), VP, P(VP)]),
        "mpm_batch_destroy": (I32, [VP]),
        "mpm_set_particles": (I32, [VP, I32, VP, VP, VP, VP, I64]),
        "mpm_get_particles": (I32, [VP, I32, VP, VP, VP, VP]),
        "mpm_set_material": (I32, [VP, I32, I32, D8]),
        "mpm_set_box_collider": (I32, [VP, I32, F3, F3, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_set_sphere_collider": (I32, [VP, I32, F3, ctypes.c_float, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_set_rounded_box_collider": (I32, [VP, I32, F3, F3, ctypes.c_float, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_forward": (I32, [VP, I32, I32]),
        "mpm_backward": (I32, [VP, VP, VP, VP, VP, VP, VP, VP, VP, VP]),
        "mpm_autotune": (I32, [VP, I32]),
        "mpm_sync": (I32, [VP]),
        "mpm_env_errors": (I32, [VP, P(I32)]),
        "mpm_memory_bytes": (I64, [VP]),
        "mpm_kernel_time": (I32, [VP, I32, P(ctypes.c_double)]),
        "mpm_set_timing": (I32, [VP, I32]),
        "mpm_last_error": (ctypes.c_char_p, [VP]),
        "mpm_version": (ctypes.c_char_p, []),
        "mpm_sort_keys": (I32, [VP, VP, VP, VP, P(I32)]),
        "mpm_set_option": (I32, [VP, I32, I32]),
        "mpm_get_option": (I32, [VP, I32, P(I32)]),
        "mpm_forward_envs": (I32, [VP, P(I32), I32]),
        "mpm_configure_env": (I32, [VP, I32, P(mpm_env_desc)]),
        "mpm_set_collider_motion": (I32, [VP, I32, F3, F3, I32]),
        "mpm_get_collider_grad": (I32, [VP, I32, D8, D8, D8, D8, I32]),
        "mpm_set_box_rotation": (I32, [VP, I32, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_set_collider": (I32, [VP, I32, I32, I32, F3, F3, ctypes.c_float, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_set_collider_rotation": (I32, [VP, I32, I32, F3, ctypes.c_float, ctypes.c_float]),
        "mpm_set_collider_motion_at": (I32, [VP, I32, I32, F3, F3, I32]),
        "mpm_get_collider_grad_at": (I32, [VP, I32, I32, D8, D8, D8, D8, I32]),
        "mpm_moments": (I32, [VP, VP, VP, VP, VP]),
        "mpm_moments_vjp": (I32, [VP, VP, VP, VP, VP, VP, VP]),
        "mpm_server_create": (I32, [P(mpm_server_desc), P(mpm_allocator), VP, P(VP)]),
        "mpm_server_destroy": (I32, [VP]),
        "mpm_server_submit": (I32, [VP, P(mpm_request), P(I64)]),
        "mpm_server_step": (I32, [VP]),
        "mpm_server_poll": (I32, [VP, I64, P(mpm_request_status)]),
        "mpm_server_cancel": (I32, [VP, I64]),
        "mpm_server_now": (ctypes.c_double, [VP]),
        "mpm_server_idle": (I32, [VP]),
        "mpm_server_stats_get": (I32, [VP, P(mpm_server_stats)]),
        "mpm_server_last_error": (ctypes.c_char_p, [VP]),
        "mpm_sort_keys_noalloc": (I32, [VP, I64, I32, VP, VP, VP]),
        "mpm_pair_distance": (I32, [VP, VP, VP, I64, VP]),
        "mpm_pair_distance_vjp": (I32, [VP, VP, VP, I64, VP, VP, VP]),
        "mpm_fem_create": (I32, [P(mpm_fem_desc), P(I32), P(mpm_allocator), VP, P(VP)]),
        "mpm_fem_destroy": (I32, [VP]),
        "mpm_fem_set_rest": (I32, [VP, VP]),
        "mpm_fem_set_params": (I32, [VP, D8]),
        "mpm_fem_set_state": (I32, [VP, VP, VP]),
        "mpm_fem_get_state": (I32, [VP, VP, VP]),
        "mpm_fem_forward": (I32, [VP, I32, VP, I32]),
        "mpm_fem_backward": (I32, [VP, VP, VP, VP, VP, VP, VP]),
        "mpm_fem_sync": (I32, [VP]),
        "mpm_fem_env_errors": (I32, [VP, P(I32)]),
        "mpm_fem_last_error": (ctypes.c_char_p, [VP]),
        "mpm_fem_memory_bytes": (I64, [VP]),
        "mpm_rb_create": (I32, [P(mpm_rb_desc), P(mpm_rb_link), P(mpm_rb_contact), P(mpm_allocator), VP, P(VP)]),
        "mpm_rb_destroy": (I32, [VP]),
        "mpm_rb_set_params": (I32, [VP, D8]),
        "mpm_rb_set_state": (I32, [VP, VP, VP]),
        "mpm_rb_get_state": (I32, [VP, VP, VP]),
        "mpm_rb_forward": (I32, [VP, I32, VP, I32]),
        "mpm_rb_backward": (I32, [VP, VP, VP, VP, VP, VP, VP]),
        "mpm_rb_sync": (I32, [VP]),
        "mpm_rb_env_errors": (I32, [VP, P(I32)]),
        "mpm_rb_last_error": (ctypes.c_char_p, [VP]),
        "mpm_rb_memory_bytes": (I64, [VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def ptr(t) -> int:
    """Device address of a tensor (None -> NULL)."""
    return None if t is None else t.data_ptr()


class MPMError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({msg})")
        self.code = code


def check(code: int, where: str, handle=None, server: bool = False, fem: bool = False, rb: bool = False):
    if code != MPM_OK:
        msg = ""
        if _lib is not None:
            err = (_lib.mpm_server_last_error if server else _lib.mpm_fem_last_error if fem else
                   _lib.mpm_rb_last_error if rb else _lib.mpm_last_error)
            raw = err(handle)
            msg = raw.decode() if raw else ""
        raise MPMError(code, where, msg)
    return code
