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
FLAG_NAN, FLAG_POSINF, FLAG_ALL_NEGINF, FLAG_BAD_ANCESTOR, FLAG_INTERNAL = 1, 2, 4, 8, 16
STRATIFIED, SYSTEMATIC, MULTINOMIAL, METROPOLIS, LOG_SUM_EXP = 0, 1, 2, 3, 4


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("lds_max_p", ctypes.c_int64), ("lanes_per_chain", ctypes.c_int32)]


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
        "rs_workspace_bytes": (sz, [i64, ctypes.c_int]),
        "rs_workspace_init": (ctypes.c_int, [vp, sz, vp]),
        "resample_metropolis": (ctypes.c_int, [vp, vp, i64, u32, u64, u32, i32p, vp]),
        "resample_stratified": (ctypes.c_int, [vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "resample_systematic": (ctypes.c_int, [vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "resample_multinomial": (ctypes.c_int, [vp, vp, i64, u64, u32, vp, vp, sz, i32p, vp]),
        "ancestors_to_offspring": (ctypes.c_int, [vp, vp, i64, i32p, vp]),
        "permute_copy": (ctypes.c_int, [vp, vp, vp, i64, ctypes.c_int32, i32p, vp]),
        "rs_log_sum_exp": (ctypes.c_int, [vp, i64, vp, vp, sz, i32p, vp]),
        "metropolis_B": (u32, [i64, ctypes.c_double, ctypes.c_double]),
        "rs_log_u_table": (ctypes.c_int, [vp, vp, vp]),
        "rs_metropolis_set_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
        "rs_metropolis_get_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
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
        raise ResampleError(f"{what}: {lib.rs_strerror(rc).decode()} (rc={rc})")
    return rc
