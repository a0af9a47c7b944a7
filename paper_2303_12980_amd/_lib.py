"""ctypes declarations of the C ABI in include/gmp.h (argument marshalling
only; every step of the feature path runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmp.so")

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P_i32 = ctypes.POINTER(c_i32)
P_dbl = ctypes.POINTER(c_dbl)

GMP_OK, GMP_E_INVALID, GMP_E_UNSUPPORTED, GMP_E_CELL = 0, 1, 2, 3
GMP_E_CAPACITY, GMP_E_NONFINITE, GMP_E_HIP, GMP_E_NOMEM, GMP_E_STALE = 4, 5, 6, 7, 8
STATUS_NAMES = {0: "GMP_OK", 1: "GMP_E_INVALID", 2: "GMP_E_UNSUPPORTED", 3: "GMP_E_CELL",
                4: "GMP_E_CAPACITY", 5: "GMP_E_NONFINITE", 6: "GMP_E_HIP", 7: "GMP_E_NOMEM", 8: "GMP_E_STALE"}
GMP_FP64, GMP_FP32_COMPENSATED, GMP_FP32_WIDE = 0, 1, 2

# every symbol include/gmp.h declares
EXPORTS = (
    "gmp_probe_cutoffs", "gmp_plan_create", "gmp_plan_destroy", "gmp_plan_info", "gmp_plan_get_tuning", "gmp_plan_set_tuning",
    "gmp_workspace_size", "gmp_build_neighbors", "gmp_build_lists", "gmp_build_reverse", "gmp_features",
    "gmp_features_noalloc", "gmp_features_backward", "gmp_feature_jacobian",
    "gmp_check_status", "gmp_profile_begin", "gmp_profile_end", "gmp_last_error",
)


class ProbeDesc(ctypes.Structure):
    _fields_ = [("n_orders", c_i32), ("orders", P_i32), ("n_sigmas", c_i32), ("sigmas", P_dbl),
                ("n_elements", c_i32), ("prim_offsets", P_i32), ("B", P_dbl), ("beta", P_dbl),
                ("overlap_threshold", c_dbl), ("screening", c_i32), ("radial_intervals", c_i32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_structs", c_i32), ("n_atoms", c_i64), ("atom_offsets", c_vp), ("x", c_vp), ("y", c_vp),
                ("z", c_vp), ("species", c_vp), ("cell", c_vp), ("pbc", c_vp), ("occupancy", c_vp),
                ("n_points", c_i64), ("point_offsets", c_vp), ("px", c_vp), ("py", c_vp), ("pz", c_vp)]


class NbrDesc(ctypes.Structure):
    _fields_ = [("capacity", c_i64), ("n_pairs", c_i64), ("offsets", c_vp), ("j", c_vp), ("shift", c_vp),
                ("bucket_start", c_vp), ("sigma_end", c_vp), ("wrap", c_vp), ("rw", c_vp), ("reverse", c_vp),
                ("max_list", c_i64), ("order", c_vp), ("slot", c_vp)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_pairs", c_i32), ("bin_divisor", c_i32), ("blocks_per_cu", c_i32), ("adj_items", c_i32),
                ("sigma_groups", c_i32)]


class GMPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libgmp.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2303_12980_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    L.gmp_plan_create.argtypes = [ctypes.POINTER(ProbeDesc), c_i32, ctypes.POINTER(c_vp)]
    L.gmp_plan_create.restype = c_i32
    L.gmp_probe_cutoffs.argtypes = [ctypes.POINTER(ProbeDesc), P_dbl]
    L.gmp_probe_cutoffs.restype = c_i32
    L.gmp_plan_destroy.argtypes = [c_vp]
    L.gmp_plan_destroy.restype = None
    L.gmp_plan_info.argtypes = [c_vp, P_i32, P_i32, P_i32, P_dbl]
    L.gmp_plan_info.restype = c_i32
    L.gmp_plan_get_tuning.argtypes = [c_vp, ctypes.POINTER(Tuning)]
    L.gmp_plan_get_tuning.restype = c_i32
    L.gmp_plan_set_tuning.argtypes = [c_vp, ctypes.POINTER(Tuning)]
    L.gmp_plan_set_tuning.restype = c_i32
    L.gmp_workspace_size.argtypes = [c_vp, c_i32, c_i64, c_i64, c_i64, ctypes.POINTER(ctypes.c_size_t)]
    L.gmp_workspace_size.restype = c_i32
    L.gmp_build_neighbors.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc),
                                      ctypes.POINTER(c_i64), c_vp, ctypes.c_size_t, c_vp]
    L.gmp_build_neighbors.restype = c_i32
    L.gmp_build_lists.argtypes = L.gmp_build_neighbors.argtypes
    L.gmp_build_lists.restype = c_i32
    L.gmp_build_reverse.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc), c_vp, ctypes.c_size_t,
                                    c_vp]
    L.gmp_build_reverse.restype = c_i32
    L.gmp_features.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc), c_vp, c_vp, c_vp,
                               ctypes.c_size_t, c_vp]
    L.gmp_features.restype = c_i32
    L.gmp_features_noalloc.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc), c_vp, c_vp, c_vp]
    L.gmp_features_noalloc.restype = c_i32
    L.gmp_features_backward.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc), c_vp, c_vp,
                                        c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]
    L.gmp_features_backward.restype = c_i32
    L.gmp_feature_jacobian.argtypes = [c_vp, ctypes.POINTER(BatchDesc), ctypes.POINTER(NbrDesc), c_vp, c_vp, c_i64,
                                       c_vp, ctypes.c_size_t, c_vp]
    L.gmp_feature_jacobian.restype = c_i32
    L.gmp_check_status.argtypes = [c_vp, ctypes.c_size_t, c_vp]
    L.gmp_check_status.restype = c_i32
    L.gmp_profile_begin.argtypes = []
    L.gmp_profile_begin.restype = c_i32
    L.gmp_profile_end.argtypes = [c_i32, P_i32, ctypes.c_char_p, P_i32, P_dbl]
    L.gmp_profile_end.restype = c_i32
    L.gmp_last_error.argtypes = []
    L.gmp_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status):
    if status != GMP_OK:
        msg = load().gmp_last_error()
        raise GMPError(status, msg.decode() if msg else "")
    return status
