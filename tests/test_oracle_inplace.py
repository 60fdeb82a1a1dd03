"""Pins of the oracle's minimal-copy state update (offspring form, Sec. 2).

What fixes it: the resampled population is the multiset {x_j repeated o_j
times} (every particle then carries weight 1/P, so slot order is free); rows
of particles with offspring stay in their slots; each empty slot takes one
extra copy, holes and extras both in increasing order. Checked against a
hand-worked case, against an independent vectorised construction, and
against the ancestor-indexed copy of the oracle's own resamplers as a
multiset of rows.
"""
import numpy as np
import pytest

import oracle
from paper_1202_6163_amd import workloads


def rows_sorted(x, D):
    r = np.ascontiguousarray(x.reshape(-1, D)).view(np.uint32)
    return r[np.lexsort(r.T[::-1])]


def test_hand_worked_case():
    off = np.array([0, 3, 0, 1, 0, 2], dtype=np.int32)
    x = np.arange(12, dtype=np.float32).reshape(6, 2)
    xo, anc, rc = oracle.offspring_update_inplace(off, x)
    assert rc == 0
    # holes 0, 2, 4 take the extras 1, 1, 5 in order; 1, 3, 5 stay
    assert anc.tolist() == [1, 1, 1, 3, 5, 5]
    assert xo.reshape(6, 2).tolist() == [[2, 3], [2, 3], [2, 3], [6, 7], [10, 11], [10, 11]]


def vectorised(off):
    P = off.size
    extras = np.repeat(np.arange(P, dtype=np.int32), np.maximum(off - 1, 0))
    holes = np.flatnonzero(off == 0)
    anc = np.arange(P, dtype=np.int32)
    anc[holes] = extras
    return anc


@pytest.mark.parametrize("kind", ["stratified", "systematic", "multinomial", "metropolis"])
@pytest.mark.parametrize("P,sigma,D", [(1, 1.0, 3), (7, 2.0, 1), (1000, 1.0, 4), (4099, 4.0, 16)])
def test_against_resamplers(kind, P, sigma, D):
    lw = workloads.normal_logweights(P, sigma, 5)
    if kind == "metropolis":
        anc, _ = oracle.metropolis(lw, 64, 3, 0)
    else:
        anc, _ = getattr(oracle, kind)(lw, 3, 0)
    off, _ = oracle.ancestors_to_offspring(anc)
    x = workloads.state_rows_exact(P, D)
    xo, a2, rc = oracle.offspring_update_inplace(off, x)
    assert rc == 0
    # the same population as the ancestor-indexed copy
    ref, _ = oracle.permute_copy(anc, x)
    assert np.array_equal(rows_sorted(xo, D), rows_sorted(ref, D))
    # the independent construction, slot for slot
    assert np.array_equal(a2, vectorised(off))
    assert np.array_equal(np.bincount(a2, minlength=P), off)
    keep = off >= 1
    assert np.array_equal(a2[keep], np.flatnonzero(keep))
    xr, x0 = xo.reshape(P, D), x.reshape(P, D)
    assert np.array_equal(xr[keep], x0[keep])
    assert np.array_equal(xr, x0[a2])
    # only the holes changed (rows of the exact state are distinct)
    changed = np.any(xr != x0, axis=1)
    assert changed.sum() == np.count_nonzero(off == 0)
    assert np.all(np.diff(a2[off == 0]) >= 0)


def test_identity_and_concentrated():
    P, D = 513, 2
    x = workloads.state_rows_exact(P, D)
    xo, a2, rc = oracle.offspring_update_inplace(np.ones(P, dtype=np.int32), x)
    assert rc == 0 and np.array_equal(a2, np.arange(P)) and np.array_equal(xo, x)
    off = np.zeros(P, dtype=np.int32)
    off[300] = P
    xo, a2, rc = oracle.offspring_update_inplace(off, x)
    assert rc == 0 and np.all(a2 == 300)
    assert np.array_equal(xo.reshape(P, D), np.repeat(x.reshape(P, D)[300:301], P, axis=0))


@pytest.mark.parametrize("bad", ["sum_low", "sum_high", "negative"])
def test_invalid_counts_leave_state(bad):
    P, D = 100, 3
    off = np.ones(P, dtype=np.int32)
    if bad == "sum_low":
        off[5] = 0
    elif bad == "sum_high":
        off[5] = 2
    else:
        off[5], off[6] = -1, 3
    x = workloads.state_rows_exact(P, D)
    xo, a2, rc = oracle.offspring_update_inplace(off, x)
    assert rc == oracle.FLAG_BAD_ANCESTOR
    assert np.array_equal(xo, x) and np.array_equal(a2, np.arange(P))
