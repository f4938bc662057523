"""Pins for the oracle's primitives (Sec. 4 toy task and Alg. 1/2; Sec. 2 API).

select_update is pinned three ways: hand-worked toy-task vectors, exhaustive
agreement with two independent literal formulations of the paper's algorithms
(Rank-Match, Sort-Count-Iterate) over every small mask pattern, and special
cases that reduce to numpy routines.  add/remove/resolve are pinned by their
defining properties and by brute force on tiny inputs.
"""
import itertools

import numpy as np
import pytest

from conftest import golden_path


def _toy_cases():
    cases = []
    for line in open(golden_path("toy_task_vectors.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        a, b, exp, r, dropped = (f.split() for f in line.split("|"))
        cases.append(([int(v) for v in a], [int(v) for v in b], [int(v) for v in exp],
                      int(r[0]), int(dropped[0])))
    return cases


def _toy_via_select_update(orc, a, b):
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    sel = (a % 2 == 0).astype(np.uint8)
    upd = (b % 2 != 0).astype(np.uint8)
    out, applied, dropped = orc.select_update(a.astype(np.int32)[None, :], sel,
                                              b.astype(np.int32)[None, :], upd_mask=upd)
    return out[0].astype(np.int64), applied, dropped


def test_toy_task_hand_vectors(orc):
    cases = _toy_cases()
    assert len(cases) == 8
    for a, b, exp, r, dropped in cases:
        assert list(orc.toy_rank_match(a, b)) == exp, (a, b)
        assert list(orc.toy_sort_count_iterate(a, b)) == exp, (a, b)
        got, applied, drop = _toy_via_select_update(orc, a, b)
        assert list(got) == exp and applied == r and drop == dropped, (a, b)


def test_literal_rank_match_needs_positive_label_guard(orc):
    """Comparing labels without requiring them to be positive overwrites an
    unselected entry with an unselected update: a=[1,2], b=[3,4] gives [4,3]."""
    assert list(orc.toy_rank_match([1, 2], [3, 4], guard=False)) == [4, 3]
    assert list(orc.toy_rank_match([1, 2], [3, 4], guard=True)) == [1, 3]


def test_exhaustive_small_patterns_rm_sci_select_update_agree(orc):
    """Every parity pattern of a (n <= 5) and b (m <= 5): Rank-Match, Sort-Count-
    Iterate, select_update and a numpy flatnonzero formulation agree."""
    rng = np.random.default_rng(0)
    count = 0
    for n in range(0, 6):
        for m in range(0, 6):
            for pa in itertools.product((0, 1), repeat=n):
                for pb in itertools.product((0, 1), repeat=m):
                    a = rng.integers(-50, 50, size=n) * 2 + np.array(pa, dtype=np.int64)
                    b = rng.integers(-50, 50, size=m) * 2 + np.array(pb, dtype=np.int64)
                    rm = orc.toy_rank_match(a, b)
                    sci = orc.toy_sort_count_iterate(a, b)
                    su, applied, dropped = _toy_via_select_update(orc, a, b)
                    A = np.flatnonzero(a % 2 == 0)
                    B = np.flatnonzero(b % 2 != 0)
                    r = min(A.size, B.size)
                    ref = a.copy()
                    ref[A[:r]] = b[B[:r]]
                    assert np.array_equal(rm, ref) and np.array_equal(sci, ref)
                    assert np.array_equal(su, ref)
                    assert applied == r and dropped == B.size - r
                    count += 1
    assert count == 63 * 63


def test_select_indices_is_flatnonzero(orc):
    for n in range(0, 11):
        for bits in range(1 << n):
            mask = np.array([(bits >> i) & 1 for i in range(n)], dtype=np.uint8)
            assert np.array_equal(orc.select_indices(mask), np.flatnonzero(mask))
    mask = (np.random.default_rng(1).random(100000) < 0.3).astype(np.uint8) * 7
    assert np.array_equal(orc.select_indices(mask), np.flatnonzero(mask))


def _soa(rng, A, n):
    return rng.integers(-2**31, 2**31, size=(A, n), dtype=np.int64).astype(np.int32)


@pytest.mark.parametrize("p", [0.0, 0.01, 0.5, 1.0])
@pytest.mark.parametrize("q_frac", [0.0, 0.5, 1.0, 2.0])
def test_select_update_special_cases(orc, p, q_frac):
    rng = np.random.default_rng(int(p * 100) + int(q_frac * 10))
    A, n = 3, 5000
    attrs = _soa(rng, A, n)
    mask = (rng.random(n) < p).astype(np.uint8)
    k = int(mask.sum())
    q = int(q_frac * k) if p > 0 else int(q_frac * 100)
    recs = _soa(rng, A, q)
    out, applied, dropped = orc.select_update(attrs, mask, recs)
    r = min(k, q)
    assert applied == r and dropped == q - r
    sel = np.flatnonzero(mask)
    untouched = np.ones(n, dtype=bool)
    untouched[sel[:r]] = False
    assert np.array_equal(out[:, untouched], attrs[:, untouched])
    assert np.array_equal(out[:, sel[:r]], recs[:, :r])
    # idempotent: applying the same update again changes nothing
    out2, _, _ = orc.select_update(out, mask, recs)
    assert np.array_equal(out2, out)


def test_select_update_all_selected_is_a_copy(orc):
    rng = np.random.default_rng(5)
    attrs = _soa(rng, 4, 777)
    recs = _soa(rng, 4, 777)
    out, applied, dropped = orc.select_update(attrs, np.ones(777, np.uint8), recs)
    assert np.array_equal(out, recs) and applied == 777 and dropped == 0


def test_select_update_with_update_mask(orc):
    rng = np.random.default_rng(6)
    attrs, recs = _soa(rng, 2, 1000), _soa(rng, 2, 1500)
    sel = (rng.random(1000) < 0.4).astype(np.uint8)
    upd = (rng.random(1500) < 0.2).astype(np.uint8)
    out, applied, dropped = orc.select_update(attrs, sel, recs, upd_mask=upd)
    A, B = np.flatnonzero(sel), np.flatnonzero(upd)
    r = min(A.size, B.size)
    ref = attrs.copy()
    ref[:, A[:r]] = recs[:, B[:r]]
    assert np.array_equal(out, ref) and applied == r and dropped == B.size - r


@pytest.mark.parametrize("free_p,q", [(0.0, 10), (0.3, 0), (0.3, 100), (0.3, 10**6), (1.0, 50)])
def test_add_agents_fills_lowest_free_slots(orc, free_p, q):
    rng = np.random.default_rng(7)
    n = 3000
    q = min(q, 5000)
    attrs, recs = _soa(rng, 3, n), _soa(rng, 3, q)
    alive = (rng.random(n) >= free_p).astype(np.int32) * rng.integers(1, 5, size=n).astype(np.int32)
    out, al, added, dropped = orc.add_agents(attrs, alive, recs)
    F = np.flatnonzero(alive == 0)
    r = min(F.size, q)
    assert added == r and dropped == q - r
    assert np.count_nonzero(al) == np.count_nonzero(alive) + r
    assert np.all(al[F[:r]] == 1) and np.all(al[F[r:]] == 0)
    keep = np.ones(n, bool)
    keep[F[:r]] = False
    assert np.array_equal(al[keep], alive[keep])
    assert np.array_equal(out[:, F[:r]], recs[:, :r])
    assert np.array_equal(out[:, keep], attrs[:, keep])


def test_remove_agents_masked_update(orc):
    rng = np.random.default_rng(8)
    n = 4000
    alive = (rng.random(n) < 0.7).astype(np.int32)
    kill = (rng.random(n) < 0.2).astype(np.uint8) * 3
    al, removed = orc.remove_agents(alive, kill)
    assert removed == int(np.count_nonzero((kill != 0) & (alive != 0)))
    assert np.count_nonzero(al) == np.count_nonzero(alive) - removed
    assert np.all(al[kill != 0] == 0)
    assert np.array_equal(al[kill == 0], alive[kill == 0])


def _brute_resolve(targets, prios, active, n_t):
    best = {}
    for c, (t, p) in enumerate(zip(targets, prios)):
        if not active[c] or t < 0 or t >= n_t:
            continue
        if t not in best or (p, c) < best[t]:
            best[t] = (p, c)
    return best


def test_resolve_conflicts_exhaustive_small(orc):
    """Every assignment of up to 5 claimants to 3 targets (or none), every
    priority permutation, and every pattern of tied priorities."""
    n_t = 3
    cases = 0
    for n in range(0, 6):
        prio_sets = set(itertools.permutations(range(n)))
        prio_sets |= set(itertools.product((0, 1), repeat=n))  # ties
        for tg in itertools.product(range(-1, n_t), repeat=n):
            for pr in list(prio_sets)[:24]:
                active = [t >= 0 for t in tg]
                tgt = np.array([t if t >= 0 else 0 for t in tg], dtype=np.int32)
                best, winner, won = orc.resolve_conflicts(
                    tgt, np.array(pr, dtype=np.uint32), n_t, active=np.array(active, np.uint8))
                ref = _brute_resolve(list(tgt), list(pr), active, n_t)
                for t in range(n_t):
                    if t in ref:
                        p, c = ref[t]
                        assert winner[t] == c and best[t] == (p << 32) | c
                    else:
                        assert winner[t] == -1 and best[t] == 2**64 - 1
                for c in range(n):
                    exp = active[c] and ref[int(tgt[c])][1] == c
                    assert bool(won[c]) == exp
                # exactly one winner per claimed target
                assert int(won.sum()) == len(ref)
                cases += 1
    assert cases > 1000


def test_resolve_conflicts_out_of_range_targets_ignored(orc):
    tgt = np.array([0, 5, -3, 1, 1], dtype=np.int32)
    pr = np.array([9, 0, 0, 4, 2], dtype=np.uint32)
    best, winner, won = orc.resolve_conflicts(tgt, pr, 2)
    assert list(winner) == [0, 4] and list(won) == [1, 0, 0, 0, 1]
