"""ctypes view of the C ABI declared in include/abadj.h.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libabadj.so.  There is no fallback: if the library is missing
the import fails with instructions to build it.
"""
from __future__ import annotations

import ctypes
import os

from ._build import LIB

SIM_OK = 0
SIM_ERR_INVALID_ARG = -1
SIM_ERR_INVALID_TOPOLOGY = -2
SIM_ERR_WORKSPACE_TOO_SMALL = -3
SIM_ERR_UNSUPPORTED_DTYPE = -4
SIM_ERR_HIP = -5
SIM_F32 = 0
SIM_F64 = 1
SIM_JOINT_REVOLUTE = 0
SIM_JOINT_FREE = 1
SIM_JOINT_PRISMATIC = 2
SIM_JOINT_SPHERICAL = 3
SIM_MAX_LINKS = 64

EXPORTED = ("sim_create", "sim_destroy", "sim_get_info", "sim_set_adjoint_dtype", "sim_status", "sim_get_tiling",
            "sim_set_tiling", "sim_autotune", "sim_autotune_cache_clear",
            "sim_workspace_bytes",
            "sim_checkpoint_schedule", "sim_forward", "sim_forward_jvp",
            "sim_backward", "sim_backward_noalloc", "sim_aba", "sim_flops", "sim_last_error",
            "sim_pgs_workspace_bytes", "sim_pgs_solve", "sim_pgs_adjoint",
            "sim_contact_param_count", "sim_contact_flops", "sim_contact_rollout", "sim_contact_rollout_grad",
            "sim_contact_autotune")
SIM_PGS_MAX_ROWS = 16


class SimTopology(ctypes.Structure):
    _fields_ = [("n_sys", ctypes.c_int32), ("link_offset", ctypes.c_void_p),
                ("parent", ctypes.c_void_p), ("jtype", ctypes.c_void_p)]


class SimParams(ctypes.Structure):
    _fields_ = [("E_T", ctypes.c_void_p), ("r_T", ctypes.c_void_p), ("axis", ctypes.c_void_p),
                ("mass", ctypes.c_void_p), ("com", ctypes.c_void_p), ("Ic", ctypes.c_void_p),
                ("gravity", ctypes.c_void_p), ("limits", ctypes.c_void_p)]


class SimInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("n_sys", "n_links", "nq", "nv", "nu", "n_waves",
                                               "n_slots", "max_depth", "has_free", "dtype",
                                               "frames_identity", "chain", "has_prism", "adjoint_dtype",
                                               "has_ball")]


class SimTiling(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("waves_per_block", "pairs_per_block", "pipelined")]


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"abadj error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libabadj.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with `python -m paper_2109_07719_amd._build` "
                              "(or __graft_entry__.build()); there is no non-HIP fallback")
        L = ctypes.CDLL(LIB)
        P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.sim_create.argtypes = [ctypes.POINTER(SimTopology), ctypes.POINTER(SimParams), I,
                                 ctypes.POINTER(P)]
        L.sim_create.restype = I
        L.sim_destroy.argtypes = [P]
        L.sim_destroy.restype = None
        L.sim_get_info.argtypes = [P, ctypes.POINTER(SimInfo)]
        L.sim_get_info.restype = I
        L.sim_set_adjoint_dtype.argtypes = [P, I]
        L.sim_set_adjoint_dtype.restype = I
        L.sim_get_tiling.argtypes = [P, ctypes.POINTER(SimTiling)]
        L.sim_get_tiling.restype = I
        L.sim_set_tiling.argtypes = [P, ctypes.POINTER(SimTiling)]
        L.sim_set_tiling.restype = I
        L.sim_status.argtypes = [P, P, ctypes.POINTER(I)]
        L.sim_status.restype = I
        L.sim_autotune.argtypes = [P, I, I, P, ctypes.POINTER(SimTiling), ctypes.POINTER(D)]
        L.sim_autotune.restype = I
        L.sim_autotune_cache_clear.argtypes = []
        L.sim_autotune_cache_clear.restype = None
        L.sim_workspace_bytes.argtypes = [P, I, I, ctypes.POINTER(Z)]
        L.sim_workspace_bytes.restype = I
        L.sim_forward.argtypes = [P, P, P, P, D, I, I, P, P, P, P, Z, P]
        L.sim_forward.restype = I
        L.sim_backward.argtypes = [P, P, D, I, I, P, P, P, P, P, P, P, P, P, Z, P]
        L.sim_backward.restype = I
        L.sim_backward_noalloc.argtypes = [P, P, D, I, I, P, P, P, P, P, P, P, P, P, Z, P]
        L.sim_backward_noalloc.restype = I
        L.sim_pgs_workspace_bytes.argtypes = [I, I, I, I, ctypes.POINTER(Z)]
        L.sim_pgs_workspace_bytes.restype = I
        L.sim_pgs_solve.argtypes = [I, I, I, I, P, P, P, P, P, P, P, Z, P]
        L.sim_pgs_solve.restype = I
        L.sim_pgs_adjoint.argtypes = [I, I, I, I, P, P, P, P, P, P, Z, P, P, P, P, P, P]
        L.sim_pgs_adjoint.restype = I
        L.sim_checkpoint_schedule.argtypes = [I, I, P, I, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_longlong)]
        L.sim_checkpoint_schedule.restype = I
        L.sim_forward_jvp.argtypes = [P, P, P, P, P, P, P, D, I, P, P, P, P, P, P, P]
        L.sim_forward_jvp.restype = I
        L.sim_aba.argtypes = [P, P, P, P, P, P]
        L.sim_aba.restype = I
        L.sim_flops.argtypes = [P, I, ctypes.POINTER(D)]
        L.sim_flops.restype = I
        L.sim_contact_param_count.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                              ctypes.POINTER(I)]
        L.sim_contact_param_count.restype = I
        L.sim_contact_flops.argtypes = [P, P, P, P, P, D, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.sim_contact_flops.restype = I
        L.sim_contact_rollout.argtypes = [P, I, I, P, P, P, P, D, I, P, P, P, P, P]
        L.sim_contact_rollout.restype = I
        L.sim_contact_rollout_grad.argtypes = [P, I, I, P, P, P, D, I, P, P, P, P, P, P, P]
        L.sim_contact_rollout_grad.restype = I
        L.sim_contact_autotune.argtypes = [P, I, I, P, P, P, P, D, I, P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.sim_contact_autotune.restype = I
        L.sim_last_error.argtypes = []
        L.sim_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(rc: int):
    if rc != SIM_OK:
        raise SimError(rc, lib().sim_last_error().decode())
