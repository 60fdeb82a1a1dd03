"""CPU oracle for the resampling stage (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps ``liboracle.so`` (plain single-threaded C, see
``resample_oracle.c``) with numpy-level helpers, and adds the Kalman-filter
closed form in ``kalman.py``. It shares no code with the HIP library and never
imports it.

Every function takes and returns host numpy arrays.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FLAG_NAN = 1
FLAG_POSINF = 2
FLAG_ALL_NEGINF = 4
FLAG_BAD_ANCESTOR = 8

KIND_STRATIFIED = 0
KIND_SYSTEMATIC = 1
KIND_MULTINOMIAL = 2


def _load():
    src = os.path.join(_HERE, "resample_oracle.c")
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    u32, i32, i64, u64 = ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    f32p, f64p = P(ctypes.c_float), P(ctypes.c_double)
    i32p, u32p, u64p = P(i32), P(u32), P(u64)
    sig = {
        "oracle_philox4x32_10": (None, [u32p, u32p, u32p]),
        "oracle_index": (u32, [u32, i64]),
        "oracle_metropolis_u": (ctypes.c_float, [u32]),
        "oracle_log_u": (ctypes.c_float, [ctypes.c_float]),
        "oracle_log_u_table": (None, [f32p]),
        "oracle_index_histogram": (None, [i64, u64p]),
        "oracle_metropolis": (ctypes.c_int, [f32p, i32p, i64, u32, u64, u32, i32p]),
        "oracle_metropolis_many": (ctypes.c_int, [f32p, i32p, i64, u32, u64, u32, i64]),
        "oracle_metropolis_subset": (ctypes.c_int, [f32p, i64, u32, u64, u32, P(i64), i64, i32p]),
        "oracle_cumulative": (ctypes.c_int, [f32p, i64, f64p, f32p, i32p]),
        "oracle_cumulative_extended": (ctypes.c_int, [f32p, i64, f64p, f64p]),
        "oracle_search": (i64, [f64p, i64, ctypes.c_double]),
        "oracle_draw_points": (ctypes.c_int, [ctypes.c_int, i64, ctypes.c_double, u64, u32, f64p]),
        "oracle_stratified": (ctypes.c_int, [f32p, i32p, i64, u64, u32, f64p, i32p]),
        "oracle_systematic": (ctypes.c_int, [f32p, i32p, i64, u64, u32, f64p, i32p]),
        "oracle_multinomial": (ctypes.c_int, [f32p, i32p, i64, u64, u32, f64p, i32p]),
        "oracle_ancestors_to_offspring": (ctypes.c_int, [i32p, i32p, i64]),
        "oracle_offspring_to_ancestors": (ctypes.c_int, [i32p, i32p, i64]),
        "oracle_permute_copy": (ctypes.c_int, [i32p, f32p, f32p, i64, i32]),
        "oracle_offspring_update_inplace": (ctypes.c_int, [i32p, f32p, i64, i32, i32p]),
        "oracle_metropolis_B": (u32, [i64, ctypes.c_double, ctypes.c_double]),
        "oracle_resampling_error": (ctypes.c_double, [i32p, f32p, i64]),
        "oracle_filter_init": (ctypes.c_int, [f32p, i64, i32, u64]),
        "oracle_filter_step": (ctypes.c_int, [f32p, f32p, f32p, i64, i32, f64p, f32p,
                                              ctypes.c_double, ctypes.c_double, u64, u32]),
        "oracle_bootstrap_filter": (ctypes.c_int, [f64p, f32p, i32, i32, i64, ctypes.c_double,
                                                   ctypes.c_double, u64, ctypes.c_int, u32, f64p,
                                                   f32p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(rc, name):
    if rc < 0:
        raise ValueError(f"{name}: invalid arguments (rc={rc})")
    return rc


# ---------------------------------------------------------------- RNG pieces
def philox4x32_10(counter, key):
    """One Philox4x32-10 block: counter (4 u32), key (2 u32) -> 4 u32."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                              _ptr(out, ctypes.c_uint32))
    return out


def index(r, P):
    return int(_lib.oracle_index(int(r), int(P)))


def metropolis_u(r):
    return np.float32(_lib.oracle_metropolis_u(int(r)))


def log_u(u):
    return np.float32(_lib.oracle_log_u(float(u)))


def log_u_table():
    """L(u) on the whole u grid (2^23 binary32 values, grid order)."""
    out = np.empty(1 << 23, dtype=np.float32)
    _lib.oracle_log_u_table(_ptr(out, ctypes.c_float))
    return out


def index_histogram(P):
    counts = np.zeros(int(P), dtype=np.uint64)
    _lib.oracle_index_histogram(int(P), _ptr(counts, ctypes.c_uint64))
    return counts


# ---------------------------------------------------------------- resamplers
def metropolis(lw, B, seed, instance=0):
    """Metropolis ancestors for log-weights lw; returns (anc, status flags)."""
    lw = _f32(lw)
    anc = np.empty(lw.size, dtype=np.int32)
    st = np.zeros(1, dtype=np.int32)
    _check(_lib.oracle_metropolis(_ptr(lw, ctypes.c_float), _ptr(anc, ctypes.c_int32), lw.size,
                                  int(B), int(seed), int(instance), _ptr(st, ctypes.c_int32)),
           "metropolis")
    return anc, int(st[0])


def metropolis_many(lw, B, seed, inst0, n_inst):
    lw = _f32(lw)
    anc = np.empty((int(n_inst), lw.size), dtype=np.int32)
    _check(_lib.oracle_metropolis_many(_ptr(lw, ctypes.c_float), _ptr(anc, ctypes.c_int32),
                                       lw.size, int(B), int(seed), int(inst0), int(n_inst)),
           "metropolis_many")
    return anc


def metropolis_subset(lw, B, seed, instance, idx):
    """Metropolis ancestors of the particles in idx only."""
    lw = _f32(lw)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.int32)
    _check(_lib.oracle_metropolis_subset(_ptr(lw, ctypes.c_float), lw.size, int(B), int(seed),
                                         int(instance), _ptr(idx, ctypes.c_int64), idx.size,
                                         _ptr(out, ctypes.c_int32)), "metropolis_subset")
    return out


def cumulative(lw):
    """(C, m, flags): binary64 left-to-right prefix sums of exp(lw - max lw)."""
    lw = _f32(lw)
    C = np.empty(lw.size, dtype=np.float64)
    m = np.zeros(1, dtype=np.float32)
    st = np.zeros(1, dtype=np.int32)
    _lib.oracle_cumulative(_ptr(lw, ctypes.c_float), lw.size, _ptr(C, ctypes.c_double),
                           _ptr(m, ctypes.c_float), _ptr(st, ctypes.c_int32))
    return C, float(m[0]), int(st[0])


def cumulative_extended(lw):
    """Extended-precision prefix sums as (hi, lo) binary64 pairs."""
    lw = _f32(lw)
    hi = np.empty(lw.size, dtype=np.float64)
    lo = np.empty(lw.size, dtype=np.float64)
    _check(_lib.oracle_cumulative_extended(_ptr(lw, ctypes.c_float), lw.size,
                                           _ptr(hi, ctypes.c_double), _ptr(lo, ctypes.c_double)),
           "cumulative_extended")
    return hi, lo


def search(C, x):
    C = np.ascontiguousarray(C, dtype=np.float64)
    return int(_lib.oracle_search(_ptr(C, ctypes.c_double), C.size, float(x)))


def draw_points(kind, P, W, seed, instance=0):
    x = np.empty(int(P), dtype=np.float64)
    _check(_lib.oracle_draw_points(int(kind), int(P), float(W), int(seed), int(instance),
                                   _ptr(x, ctypes.c_double)), "draw_points")
    return x


def _prefix(fn, lw, seed, instance, want_cumw):
    lw = _f32(lw)
    anc = np.empty(lw.size, dtype=np.int32)
    C = np.empty(lw.size, dtype=np.float64) if want_cumw else None
    st = np.zeros(1, dtype=np.int32)
    _check(fn(_ptr(lw, ctypes.c_float), _ptr(anc, ctypes.c_int32), lw.size, int(seed),
              int(instance), _ptr(C, ctypes.c_double), _ptr(st, ctypes.c_int32)), fn.__name__)
    if want_cumw:
        return anc, int(st[0]), C
    return anc, int(st[0])


def stratified(lw, seed, instance=0, want_cumw=False):
    return _prefix(_lib.oracle_stratified, lw, seed, instance, want_cumw)


def systematic(lw, seed, instance=0, want_cumw=False):
    return _prefix(_lib.oracle_systematic, lw, seed, instance, want_cumw)


def multinomial(lw, seed, instance=0, want_cumw=False):
    return _prefix(_lib.oracle_multinomial, lw, seed, instance, want_cumw)


def sorted_order(lw):
    """Particle indices by decreasing log-weight, equal weights in index order
    (-0 and +0 are equal). The sorted-weight variants of Sec. 3 run a
    resampler on the weights in this order."""
    lw = _f32(lw)
    key = np.where(lw == 0, np.float32(0), lw).astype(np.float64)
    return np.argsort(-key, kind="stable").astype(np.int32)


def sorted_variant(kind, lw, seed, instance=0):
    """Sorted-weight variant of the stratified, systematic or multinomial
    resampler (Sec. 3: the weights are sorted before the prefix sum; the
    ancestors are mapped back to the original particle indices). Flagged
    inputs give identity ancestors, as the plain resamplers do."""
    fn = {"stratified": stratified, "systematic": systematic, "multinomial": multinomial}[kind]
    lw = _f32(lw)
    order = sorted_order(lw)
    a_s, st = fn(lw[order], seed, instance)
    if st:
        return np.arange(lw.size, dtype=np.int32), st
    return order[a_s], st


def ancestors_to_offspring(anc):
    anc = _i32(anc)
    off = np.empty(anc.size, dtype=np.int32)
    rc = _check(_lib.oracle_ancestors_to_offspring(_ptr(anc, ctypes.c_int32),
                                                   _ptr(off, ctypes.c_int32), anc.size),
                "ancestors_to_offspring")
    return off, rc


def offspring_to_ancestors(off):
    off = _i32(off)
    anc = np.empty(off.size, dtype=np.int32)
    _check(_lib.oracle_offspring_to_ancestors(_ptr(off, ctypes.c_int32),
                                              _ptr(anc, ctypes.c_int32), off.size),
           "offspring_to_ancestors")
    return anc


def permute_copy(anc, x_in):
    anc = _i32(anc)
    x_in = _f32(x_in)
    P = anc.size
    D = x_in.size // P
    out = np.zeros_like(x_in)
    rc = _check(_lib.oracle_permute_copy(_ptr(anc, ctypes.c_int32), _ptr(x_in, ctypes.c_float),
                                         _ptr(out, ctypes.c_float), P, D), "permute_copy")
    return out, rc


def offspring_update_inplace(off, x):
    """The minimal-copy update (resample_oracle.c): returns (x updated, the
    particle each slot holds afterwards, flags); x itself is not modified."""
    off = _i32(off)
    x = _f32(x).copy()
    P = off.size
    D = x.size // P
    anc = np.empty(P, dtype=np.int32)
    rc = _check(_lib.oracle_offspring_update_inplace(_ptr(off, ctypes.c_int32),
                                                     _ptr(x, ctypes.c_float), P, D,
                                                     _ptr(anc, ctypes.c_int32)),
                "offspring_update_inplace")
    return x, anc, rc


def metropolis_B(P, w_max, eps):
    return int(_lib.oracle_metropolis_B(int(P), float(w_max), float(eps)))


# ---------------------------------------------------------------- all-core build
_omp = None


def _omp_lib():
    """liboracle_omp.so: the same source built with OpenMP (CPU baseline)."""
    global _omp
    if _omp is None:
        path = _build.LIB_OMP
        src = os.path.join(_HERE, "resample_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build(openmp=True)
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        lib.oracle_metropolis.restype = ctypes.c_int
        lib.oracle_metropolis.argtypes = [P(ctypes.c_float), P(ctypes.c_int32), ctypes.c_int64,
                                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                          P(ctypes.c_int32)]
        lib.oracle_permute_copy.restype = ctypes.c_int
        lib.oracle_permute_copy.argtypes = [P(ctypes.c_int32), P(ctypes.c_float),
                                            P(ctypes.c_float), ctypes.c_int64, ctypes.c_int32]
        _omp = lib
    return _omp


def metropolis_all_cores(lw, B, seed, instance=0):
    """oracle.metropolis on every core (OpenMP over the chains; same bits)."""
    lw = _f32(lw)
    anc = np.empty(lw.size, dtype=np.int32)
    st = np.zeros(1, dtype=np.int32)
    _check(_omp_lib().oracle_metropolis(_ptr(lw, ctypes.c_float), _ptr(anc, ctypes.c_int32),
                                        lw.size, int(B), int(seed), int(instance),
                                        _ptr(st, ctypes.c_int32)), "metropolis_all_cores")
    return anc, int(st[0])


def permute_copy_all_cores(anc, x_in):
    """oracle.permute_copy on every core (OpenMP over the rows; same bits)."""
    anc = _i32(anc)
    x_in = _f32(x_in)
    P = anc.size
    D = x_in.size // P
    out = np.zeros_like(x_in)
    rc = _check(_omp_lib().oracle_permute_copy(_ptr(anc, ctypes.c_int32),
                                               _ptr(x_in, ctypes.c_float),
                                               _ptr(out, ctypes.c_float), P, D),
                "permute_copy_all_cores")
    return out, rc


def resampling_error(off, lw):
    off = _i32(off)
    lw = _f32(lw)
    return float(_lib.oracle_resampling_error(_ptr(off, ctypes.c_int32), _ptr(lw, ctypes.c_float),
                                              lw.size))


# ---------------------------------------------------------------- filter
def filter_init(P, D, seed):
    x = np.empty((int(P), int(D)), dtype=np.float32)
    _check(_lib.oracle_filter_init(_ptr(x, ctypes.c_float), int(P), int(D), int(seed)),
           "filter_init")
    return x


def filter_step(x_in, A, y_t, q, r, seed, t):
    x_in = _f32(x_in)
    P, D = x_in.shape
    A = np.ascontiguousarray(A, dtype=np.float64)
    y_t = _f32(y_t)
    x_out = np.empty_like(x_in)
    lw = np.empty(P, dtype=np.float32)
    _check(_lib.oracle_filter_step(_ptr(x_in, ctypes.c_float), _ptr(x_out, ctypes.c_float),
                                   _ptr(lw, ctypes.c_float), P, D, _ptr(A, ctypes.c_double),
                                   _ptr(y_t, ctypes.c_float), float(q), float(r), int(seed),
                                   int(t)), "filter_step")
    return x_out, lw


def bootstrap_filter(A, y, P, q, r, seed, resampler="stratified", B=0, want_state=False):
    """Log-likelihood estimate of a bootstrap filter run (and final state)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    y = _f32(y)
    T, D = y.shape
    ll = np.zeros(1, dtype=np.float64)
    xf = np.empty((int(P), D), dtype=np.float32) if want_state else None
    code = {"stratified": 0, "metropolis": 1}[resampler]
    _check(_lib.oracle_bootstrap_filter(_ptr(A, ctypes.c_double), _ptr(y, ctypes.c_float), T, D,
                                        int(P), float(q), float(r), int(seed), code, int(B),
                                        _ptr(ll, ctypes.c_double), _ptr(xf, ctypes.c_float)),
           "bootstrap_filter")
    return (float(ll[0]), xf) if want_state else float(ll[0])
