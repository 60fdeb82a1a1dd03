"""ctypes loader for libresample.so.

torch is imported first so that the library binds to the HIP runtime torch
already loaded (both carry the soname libamdhip64.so.7): streams and device
pointers from torch are then valid in the library. There is no fallback: if
the library is missing the import fails with instructions to build it.
"""
import ctypes
import os
import re

import torch  # noqa: F401  (loads the HIP runtime the library must share)

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libresample.so")
HEADER = os.path.join(ROOT, "include", "resample.h")

RS_OK, RS_EINVAL, RS_EWORKSPACE, RS_EHIP = 0, -1, -2, -3
RS_STATIC_SCRATCH_BYTES = 12 << 20  # the no-allocation entry point's array (resample.h)
FLAG_NAN, FLAG_POSINF, FLAG_ALL_NEGINF, FLAG_BAD_ANCESTOR, FLAG_INTERNAL = 1, 2, 4, 8, 16
STRATIFIED, SYSTEMATIC, MULTINOMIAL, METROPOLIS, LOG_SUM_EXP, METROPOLIS_ADAPTIVE = 0, 1, 2, 3, 4, 5
PATH_AUTO, PATH_LAUNCHES, PATH_ONEPASS = 0, 1, 2  # rs_prefix_set_path


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("lds_max_p", ctypes.c_int64), ("lanes_per_chain", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("lw", ctypes.c_void_p), ("anc", ctypes.c_void_p), ("off", ctypes.c_void_p),
                ("x_in", ctypes.c_void_p),
                ("x_out", ctypes.c_void_p), ("status", ctypes.c_void_p), ("P", ctypes.c_int64),
                ("D", ctypes.c_int32), ("kind", ctypes.c_int32), ("B", ctypes.c_uint32),
                ("instance", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("eps", ctypes.c_double)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("chains_per_item", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("lds_max_p", ctypes.c_int64), ("blocks", ctypes.c_int32)]


class BatchPlan(ctypes.Structure):
    _fields_ = [("dev", ctypes.c_void_p), ("n_instances", ctypes.c_int32),
                ("n_tile_items", ctypes.c_int32), ("n_table_items", ctypes.c_int32),
                ("n_main_items", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("chains_per_item", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lds_max_p", ctypes.c_int64),
                ("max_table_tiles", ctypes.c_int64), ("off_tile_items", ctypes.c_uint64),
                ("off_table_items", ctypes.c_uint64), ("off_main_items", ctypes.c_uint64),
                ("smem_main", ctypes.c_uint64)]


def header_functions():
    """Names of the functions include/resample.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_0-9]+\s*\*?\s*([A-Za-z_0-9]+)\s*\(", text,
                                 flags=re.M)))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1202_6163_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32p = ctypes.c_void_p, ctypes.c_void_p
    i64, u32, u64, sz = ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "rs_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "rs_version": (ctypes.c_int, []),
        "rs_last_hip_error": (ctypes.c_char_p, []),
        "rs_workspace_bytes": (sz, [i64, ctypes.c_int]),
        "rs_workspace_init": (ctypes.c_int, [vp, sz, vp]),
        "resample_metropolis": (ctypes.c_int, [vp, vp, i64, u32, u64, u32, i32p, vp]),
        "resample_stratified": (ctypes.c_int, [vp, vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "resample_metropolis_adaptive": (ctypes.c_int, [vp, vp, i64, ctypes.c_double, u32, u64,
                                                        u32, vp, sz, vp, i32p, vp]),
        "resample_systematic": (ctypes.c_int, [vp, vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "resample_multinomial": (ctypes.c_int, [vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "resample_prefix_static": (ctypes.c_int, [ctypes.c_int, vp, vp, vp, i64, u64, u32, vp,
                                                  i32p, vp]),
        "ancestors_to_offspring": (ctypes.c_int, [vp, vp, i64, i32p, vp]),
        "rs_offspring_workspace_bytes": (sz, [i64]),
        "ancestors_to_offspring_ws": (ctypes.c_int, [vp, vp, i64, vp, sz, i32p, vp]),
        "resample_and_copy": (ctypes.c_int, [ctypes.c_int, vp, vp, vp, i64, u32, u64, u32, vp, vp,
                                             ctypes.c_int32, vp, sz, i32p, vp]),
        "rs_sorted_workspace_bytes": (sz, [i64, ctypes.c_int]),
        "rs_workspace_log_sum_exp": (ctypes.c_int, [vp, i64, vp, vp]),
        "resample_sorted": (ctypes.c_int, [ctypes.c_int, vp, vp, i64, u64, u32, vp, sz, i32p, vp]),
        "permute_copy": (ctypes.c_int, [vp, vp, vp, i64, ctypes.c_int32, i32p, vp]),
        "rs_log_sum_exp": (ctypes.c_int, [vp, i64, vp, vp, sz, i32p, vp]),
        "metropolis_B": (u32, [i64, ctypes.c_double, ctypes.c_double]),
        "rs_log_u_table": (ctypes.c_int, [vp, vp, vp]),
        "rs_probe_gather": (ctypes.c_int, [vp, i64, i64, i64, u32, vp, vp]),
        "rs_probe_philox": (ctypes.c_int, [u64, i64, i64, vp, vp]),
        "filter_init": (ctypes.c_int, [vp, i64, ctypes.c_int32, u64, vp]),
        "filter_loglik": (ctypes.c_int, [vp, ctypes.c_int32, i64, vp, vp]),
        "filter_init_batch": (ctypes.c_int, [vp, ctypes.c_int32, i64, ctypes.c_int32, u64, vp]),
        "filter_propagate_weight_batch": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, i64,
                                                         ctypes.c_int32, vp, vp, vp,
                                                         ctypes.c_double, u64, u32, vp]),
        "resample_batch_at": (ctypes.c_int, [ctypes.POINTER(BatchPlan), u32, vp]),
        "rs_batch_log_mean_weight": (ctypes.c_int, [ctypes.POINTER(BatchPlan), vp, vp]),
        "rs_batch_iterations": (ctypes.c_int, [ctypes.POINTER(BatchPlan), vp, vp]),
        "filter_propagate_weight": (ctypes.c_int, [vp, vp, vp, i64, ctypes.c_int32, vp, vp,
                                                   ctypes.c_double, ctypes.c_double, u64, u32,
                                                   vp]),
        "rs_metropolis_set_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
        "rs_batch_plan_bytes": (sz, [ctypes.POINTER(Instance), ctypes.c_int32,
                                     ctypes.POINTER(BatchTuning)]),
        "rs_batch_workspace_bytes": (sz, [ctypes.POINTER(Instance), ctypes.c_int32]),
        "rs_batch_plan_init": (ctypes.c_int, [ctypes.POINTER(BatchPlan), ctypes.POINTER(Instance),
                                              ctypes.c_int32, ctypes.POINTER(BatchTuning), vp, sz,
                                              vp, sz, vp, vp]),
        "resample_batch": (ctypes.c_int, [ctypes.POINTER(BatchPlan), vp]),
        "rs_metropolis_get_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
        "rs_prefix_set_path": (ctypes.c_int, [ctypes.c_int, i64]),
        "rs_inplace_workspace_bytes": (sz, [i64]),
        "offspring_update_inplace": (ctypes.c_int, [vp, vp, i64, ctypes.c_int32, vp, vp, sz,
                                                    i32p, vp]),
        "rs_prefix_get_path": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class ResampleError(RuntimeError):
    pass


def check(rc, what):
    if rc != RS_OK:
        detail = f" [{lib.rs_last_hip_error().decode()}]" if rc == RS_EHIP else ""
        raise ResampleError(f"{what}: {lib.rs_strerror(rc).decode()} (rc={rc}){detail}")
    return rc
