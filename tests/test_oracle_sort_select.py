"""Pins for the oracle's sort_agents and select_agents (Sec. 2 API list).

sort_agents reorders a collection by a runtime key, ascending or descending,
keeping equal keys in index order; select_agents puts the indices that satisfy
a condition first.  Pinned against numpy's stable argsort (a separate
implementation from the oracle's qsort with an index tie-break), hand-worked
cases, and the special cases that make stability visible."""
import itertools

import numpy as np
import pytest


def test_hand_worked_sort(orc):
    # keys 3 1 3 0 1 -> ascending, stable: idx 3 (0), 1 (1), 4 (1), 0 (3), 2 (3)
    key = np.array([3, 1, 3, 0, 1], dtype=np.int32)
    attrs = np.array([[10, 11, 12, 13, 14], [20, 21, 22, 23, 24]], dtype=np.int32)
    out, al, perm = orc.sort_agents(attrs, key, alive=np.array([1, 0, 1, 1, 0]))
    assert list(perm) == [3, 1, 4, 0, 2]
    assert list(out[0]) == [13, 11, 14, 10, 12] and list(out[1]) == [23, 21, 24, 20, 22]
    assert list(al) == [1, 0, 0, 1, 1]
    # descending keeps index order among equals: 0 (3), 2 (3), 1 (1), 4 (1), 3 (0)
    _, _, perm = orc.sort_agents(attrs, key, descending=True)
    assert list(perm) == [0, 2, 1, 4, 3]


@pytest.mark.parametrize("descending", [False, True])
def test_sort_matches_numpy_stable_argsort(orc, descending):
    g = np.random.default_rng(3)
    for n, lo, hi in ((1, 0, 5), (17, -3, 3), (500, -2 ** 31, 2 ** 31 - 1), (4096, 0, 16),
                      (3000, -100, 100)):
        key = g.integers(lo, hi, size=n, endpoint=True, dtype=np.int64).astype(np.int32)
        attrs = g.integers(-2 ** 31, 2 ** 31, size=(3, n), dtype=np.int64).astype(np.int32)
        exp = np.argsort(-key.astype(np.int64) if descending else key, kind="stable")
        out, _, perm = orc.sort_agents(attrs, key, descending=descending)
        assert np.array_equal(perm, exp)
        assert np.array_equal(out, attrs[:, exp])


def test_sort_special_cases(orc):
    n = 64
    attrs = np.arange(n, dtype=np.int32)[None, :]
    ident = np.arange(n)
    for key in (np.zeros(n), np.arange(n)):                         # equal keys; sorted keys
        _, _, perm = orc.sort_agents(attrs, key.astype(np.int32))
        assert np.array_equal(perm, ident)
    _, _, perm = orc.sort_agents(attrs, np.arange(n, dtype=np.int32)[::-1].copy())
    assert np.array_equal(perm, ident[::-1])
    _, _, perm = orc.sort_agents(attrs, np.zeros(n, dtype=np.int32), descending=True)
    assert np.array_equal(perm, ident)                               # stable when descending too
    ext = np.array([2 ** 31 - 1, -2 ** 31, 0, -1, 1], dtype=np.int32)
    _, _, perm = orc.sort_agents(np.zeros((1, 5), np.int32), ext)
    assert list(ext[perm]) == [-2 ** 31, -1, 0, 1, 2 ** 31 - 1]


def test_select_agents_every_small_condition(orc):
    for n in range(0, 9):
        for bits in itertools.product([0, 1], repeat=n):
            cond = np.array(bits, dtype=np.uint8)
            order, p = orc.select_agents(cond)
            assert p == int(cond.sum())
            assert np.array_equal(order, np.argsort(1 - cond.astype(np.int64), kind="stable"))


def test_select_agents_hand_worked(orc):
    order, p = orc.select_agents(np.array([0, 1, 1, 0, 1, 0], dtype=np.uint8))
    assert p == 3 and list(order) == [1, 2, 4, 0, 3, 5]
