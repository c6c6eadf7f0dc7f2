"""ctypes binding of libwpm.so (include/wpm.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwpm.so")

WPM_OK, WPM_EINVAL, WPM_ECAP, WPM_EKMAX, WPM_EHIP, WPM_ELIMIT = 0, -1, -2, -3, -4, -5
SCHED_PLAIN, SCHED_STATIC, SCHED_DYNAMIC, SCHED_PACKED = 0, 1, 2, 3
FLAG_ACCUMULATE = 1
CX_FULL_PICARD, CX_SEED = 1, 2
TOTAL_WORDS = 4
MAX_ROW_WORDS = 160
LANE_WINDOW = 512
MAX_K = 64

c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_f32p = ctypes.POINTER(ctypes.c_float)


MAX_BLOCKS, MAX_CHOICES = 16, 40


class Blocks(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("free_dims", ctypes.c_int32),
                ("num_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ridge", ctypes.c_int32 * MAX_BLOCKS), ("size", ctypes.c_uint8 * MAX_BLOCKS),
                ("count", ctypes.c_uint8 * MAX_BLOCKS),
                ("choice", (ctypes.c_uint8 * MAX_CHOICES) * MAX_BLOCKS),
                ("log2_vectors", ctypes.c_double)]


class InstanceInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in
                ("n", "m", "M", "N", "k", "W", "n_crit", "groups", "slots", "n_filter",
                 "row_words", "max_facets", "n_deferred")] + [
        ("table_words", ctypes.c_int64),
        ("filter_pass", ctypes.c_double),
        ("full_pass", ctypes.c_double),
        ("features", ctypes.c_float * 16),
    ]


class Item(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_uint32), ("cbits", ctypes.c_uint16),
                ("lanes", ctypes.c_uint16), ("first", ctypes.c_uint64)]


class Batch(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("max_row_words", ctypes.c_int32),
                ("max_groups", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("max_words", ctypes.c_int32), ("max_kp", ctypes.c_int32),
                ("d_tables", ctypes.c_void_p), ("d_offsets", ctypes.c_void_p),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Sched(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("d_items", ctypes.c_void_p),
                ("h_items", ctypes.c_void_p), ("num_items", ctypes.c_int64),
                ("d_scratch", ctypes.c_void_p), ("d_item_times", ctypes.c_void_p),
                ("d_bin_offsets", ctypes.c_void_p), ("waves_per_simd", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class HostInstance(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("k", ctypes.c_int32),
                ("facets", ctypes.c_void_p), ("basis", ctypes.c_void_p),
                ("offset", ctypes.c_void_p)]


MAX_PROPS, MAX_CLASSES = 8, 32


class Conditions(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_void_p), ("num_props", ctypes.c_int32),
                ("prop_c0", ctypes.c_void_p), ("prop_classes", ctypes.c_void_p),
                ("class_weight", ctypes.c_void_p), ("class_mask", ctypes.c_void_p),
                ("max_groups", ctypes.c_int32)]


_lib = None


class WpmError(RuntimeError):
    def __init__(self, call: str, status: int):
        L = lib()
        msg = L.wpm_strerror(status).decode()
        if status == WPM_EHIP:
            msg += ": " + L.wpm_last_hip_error().decode()
        super().__init__(f"{call} failed with status {status} ({msg})")
        self.status = status


def lib():
    """Load libwpm.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                          "or python paper_2301_00806_amd/build.py")
    # PyTorch supplies the process's HIP runtime: torch's bundled
    # libamdhip64 carries the soname libamdhip64.so.7, so once torch is loaded
    # libwpm.so binds to that same runtime (one runtime, shared streams and
    # device memory).  Loading libwpm.so first would bring in a second HIP
    # runtime from /opt/rocm and torch would then find no devices.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.wpm_strerror.restype = ctypes.c_char_p
    L.wpm_strerror.argtypes = [ctypes.c_int]
    L.wpm_last_hip_error.restype = ctypes.c_char_p
    L.wpm_last_hip_error.argtypes = []
    L.wpm_build_candidates.restype = ctypes.c_int
    L.wpm_build_candidates.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, c_u32p, ctypes.c_int32, c_i32p]
    L.wpm_kernel_basis.restype = ctypes.c_int
    L.wpm_kernel_basis.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, ctypes.c_int32, c_u32p,
                                   ctypes.c_int32, c_i32p, c_u32p, ctypes.c_int32, c_i32p]
    L.wpm_ubt_bound.restype = ctypes.c_int64
    L.wpm_ubt_bound.argtypes = [ctypes.c_int]
    L.wpm_pack_instance.restype = ctypes.c_int
    L.wpm_pack_instance.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, ctypes.c_int32, c_u32p,
                                    ctypes.c_int32, ctypes.POINTER(Blocks),
                                    ctypes.POINTER(Conditions), ctypes.c_int32,
                                    ctypes.c_uint64, c_u32p, ctypes.c_int64,
                                    ctypes.POINTER(InstanceInfo)]
    L.wpm_complex_filters.restype = ctypes.c_int
    L.wpm_complex_filters.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, c_i64p, c_u32p,
                                      ctypes.POINTER(ctypes.c_uint8)]
    L.wpm_iso_classes.restype = ctypes.c_int
    L.wpm_iso_classes.argtypes = [ctypes.c_int, ctypes.c_int64, c_i64p, c_u32p, c_i64p, c_i64p]
    L.wpm_idcm_orbits.restype = ctypes.c_int
    L.wpm_idcm_orbits.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, ctypes.c_int64, c_i64p]
    L.wpm_facet_conditions.restype = ctypes.c_int
    L.wpm_facet_conditions.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, ctypes.c_int32, c_u32p,
                                       ctypes.c_int32, c_u32p, c_u32p, c_u32p, c_i32p, c_u32p,
                                       c_i32p]
    L.wpm_convenient_basis.restype = ctypes.c_int
    L.wpm_convenient_basis.argtypes = [ctypes.c_int, ctypes.c_int, c_u32p, ctypes.c_int32, c_u32p,
                                       ctypes.c_int32, ctypes.c_int32, c_u32p,
                                       ctypes.POINTER(Blocks)]
    L.wpm_build_queue.restype = ctypes.c_int
    L.wpm_build_queue.argtypes = [c_i32p, c_f32p, c_i32p, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.POINTER(Item), ctypes.c_int64, c_i64p, c_i64p]
    L.wpm_build_pruned_queue.restype = ctypes.c_int
    L.wpm_build_pruned_queue.argtypes = [ctypes.POINTER(Blocks), c_f32p, c_i32p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Item),
                                         ctypes.c_int64, c_i64p, c_i64p]
    L.wpm_pack_bins.restype = ctypes.c_int
    L.wpm_pack_bins.argtypes = [ctypes.POINTER(Item), ctypes.c_int64, c_f32p, ctypes.c_int32,
                                ctypes.POINTER(Item), c_i64p, ctypes.POINTER(ctypes.c_double)]
    L.wpm_enumerate.restype = ctypes.c_int
    L.wpm_enumerate.argtypes = [ctypes.POINTER(Batch), ctypes.POINTER(Sched), ctypes.c_void_p,
                                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p]
    L.wpm_enumerate_noalloc.restype = ctypes.c_int
    L.wpm_enumerate_noalloc.argtypes = L.wpm_enumerate.argtypes
    L.wpm_persistent_grid.restype = ctypes.c_int
    L.wpm_persistent_grid.argtypes = [ctypes.POINTER(Batch), ctypes.c_int32, c_i32p]
    L.wpm_valu_probe.restype = ctypes.c_int
    L.wpm_valu_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.wpm_device_query.restype = ctypes.c_int
    L.wpm_device_query.argtypes = [c_i32p, c_i64p, c_i32p]
    L.wpm_collect.restype = ctypes.c_int
    L.wpm_collect.argtypes = [ctypes.POINTER(HostInstance), ctypes.c_int32, ctypes.c_void_p,
                              ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, c_u64p,
                              c_u32p, ctypes.c_int64, c_i64p, c_i64p, ctypes.c_void_p]
    vp = ctypes.c_void_p
    L.wpm_mlp_work_floats.restype = ctypes.c_int64
    L.wpm_mlp_work_floats.argtypes = [ctypes.c_int32]
    L.wpm_mlp_forward.restype = ctypes.c_int
    L.wpm_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp]
    L.wpm_mlp_grad.restype = ctypes.c_int
    L.wpm_mlp_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp]
    L.wpm_mlp_adam.restype = ctypes.c_int
    L.wpm_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
    _lib = L
    return L


def check(call: str, status: int, ok=(WPM_OK,)) -> int:
    if status not in ok:
        raise WpmError(call, status)
    return status


# Every symbol include/wpm.h declares.
EXPORTED = ("wpm_strerror", "wpm_last_hip_error", "wpm_build_candidates", "wpm_kernel_basis",
            "wpm_ubt_bound", "wpm_convenient_basis", "wpm_facet_conditions", "wpm_idcm_orbits",
            "wpm_complex_filters", "wpm_iso_classes", "wpm_pack_instance", "wpm_build_queue",
            "wpm_build_pruned_queue", "wpm_pack_bins", "wpm_enumerate", "wpm_enumerate_noalloc",
            "wpm_device_query", "wpm_persistent_grid", "wpm_valu_probe", "wpm_collect", "wpm_mlp_work_floats", "wpm_mlp_forward",
            "wpm_mlp_grad", "wpm_mlp_adam")
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS, MLP_NORM = 16, 64, 2, 5378, 36
