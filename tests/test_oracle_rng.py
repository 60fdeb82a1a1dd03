"""Pins for the oracle's random-number pieces (CPU only).

- Philox4x32-10 against rocRAND's independent open-source implementation.
- L(u) = RN32(ln u) against an 80-bit extended-precision logarithm on every
  point of the u grid.
- The index map against the exact word counts a uniform map must have.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    exe = tmp_path_factory.mktemp("pin") / "rocrand_philox_pin"
    src = os.path.join(HERE, "pins", "rocrand_philox_pin.cpp")
    subprocess.run([hipcc, "-O1", src, "-o", str(exe)], check=True, capture_output=True)
    return str(exe)


def test_philox_matches_rocrand(rocrand_pin):
    rng = np.random.default_rng(7)
    cases = [(0, 0, 0, 0, 0), (1, 0, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1, 2**32 - 1),
             (1, 5, 0, 3, 1), (12345678901234, 1023, 7, 15, 4)]
    for _ in range(300):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        c = [int(v) for v in rng.integers(0, 2**32, size=4)]
        cases.append((seed, *c))
    inp = "".join(f"{s} {a} {b} {c} {d}\n" for s, a, b, c, d in cases)
    out = subprocess.run([rocrand_pin], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for (seed, a, b, c, d), want in zip(cases, ref):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = tuple(int(v) for v in oracle.philox4x32_10([a, b, c, d], key))
        assert got == want, (seed, a, b, c, d)


def test_log_u_correctly_rounded_on_whole_grid():
    m = np.arange(1 << 23, dtype=np.int64)
    u = ((2 * m + 1).astype(np.float32) * np.float32(2.0**-24)).astype(np.float32)
    # u is exact: odd 24-bit integers times a power of two
    assert np.all(u.astype(np.float64) == (2 * m + 1) * 2.0**-24)
    ref = np.log(u.astype(np.longdouble)).astype(np.float32)
    got = oracle.log_u_table()
    mism = np.flatnonzero(got.view(np.uint32) != ref.view(np.uint32))
    assert mism.size == 0, f"{mism.size} grid points differ, first at m={mism[:5]}"
    # every value is negative: a move to an equal weight is always accepted
    assert np.all(got < 0)


def test_metropolis_u_grid_endpoints():
    assert oracle.metropolis_u(0) == np.float32(2.0**-24)
    assert oracle.metropolis_u(0xFFFFFFFF) == np.float32(1.0 - 2.0**-24)
    assert oracle.metropolis_u(511) == np.float32(2.0**-24)  # low 9 bits dropped
    assert oracle.metropolis_u(512) == np.float32(3 * 2.0**-24)


@pytest.mark.slow
def test_index_map_exhaustive_counts():
    # A uniform map of the 2^32 words onto [0, P) gives every index either
    # floor(2^32 / P) or ceil(2^32 / P) words.
    P = 6
    counts = oracle.index_histogram(P).astype(np.int64)
    assert counts.sum() == 2**32
    lo, hi = 2**32 // P, -(-2**32 // P)
    assert np.all((counts == lo) | (counts == hi))


def test_index_map_power_of_two_is_exact_and_ordered():
    # For P = 2^k the index is the top k bits of the word.
    rng = np.random.default_rng(3)
    for k in (1, 4, 10, 20, 31):
        for r in rng.integers(0, 2**32, size=50):
            assert oracle.index(int(r), 1 << k) == int(r) >> (32 - k)
    # monotone in r, and r = 2^32 - 1 maps to P - 1
    for P in (3, 1000, 2**31 - 1):
        assert oracle.index(2**32 - 1, P) == P - 1
        assert oracle.index(0, P) == 0
