"""The all-core (OpenMP) build of the oracle returns the single-threaded
oracle's bits: Metropolis chains and copied rows are independent per
particle, so splitting the particle loop across threads changes nothing."""
import os

import numpy as np

import oracle


def test_openmp_build_matches_single_thread():
    rng = np.random.default_rng(5)
    for P, B in ((1, 4), (7, 9), (4099, 33), (20000, 8)):
        lw = (rng.standard_normal(P) * 1.5).astype(np.float32)
        lw[rng.integers(0, P)] = -np.inf
        a1, s1 = oracle.metropolis(lw, B, 3, 2)
        a2, s2 = oracle.metropolis_all_cores(lw, B, 3, 2)
        assert s1 == s2 and np.array_equal(a1, a2), P
        x = rng.standard_normal((P, 5)).astype(np.float32)
        x1, r1 = oracle.permute_copy(a1, x)
        x2, r2 = oracle.permute_copy_all_cores(a1, x)
        assert r1 == r2 and np.array_equal(x1.view(np.uint32), x2.view(np.uint32))
    # a bad ancestor is flagged by both builds
    anc = np.array([0, 5, 1], dtype=np.int32)
    x = np.ones((3, 2), dtype=np.float32)
    assert oracle.permute_copy(anc, x)[1] == oracle.permute_copy_all_cores(anc, x)[1] != 0


def test_openmp_build_uses_several_threads():
    # the baseline reports its thread count; the library must be an OpenMP build
    import ctypes
    lib = oracle._omp_lib()
    assert os.path.basename(lib._name) == "liboracle_omp.so"
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_get_max_threads.restype = ctypes.c_int
    assert gomp.omp_get_max_threads() >= 1
