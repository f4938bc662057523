"""GPU parity of the select/update primitives against the CPU oracle.

Every comparison is element by element and bit-exact (all state is integer):
the full attribute arrays, alive arrays, index lists and the device counts.
Sizes span empty inputs, sub-wave and sub-tile sizes, several 4096-slot tiles
with a ragged tail, and the full 2^24-slot x 8-attribute microbenchmark at
the densities p in {0.001, 0.05, 0.5} for seeds 0-9.
"""
import numpy as np
import pytest
import torch

from paper_2508_16508_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 63, 64, 65, 1000, 4095, 4096, 4097, 4096 + 3000, 3 * 4096 + 77, 100_003]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _run_select(abm, attrs, mask, recs, upd_mask=None, ws=None):
    d_attrs = dev(attrs)
    applied, dropped = abm.select_update(d_attrs, dev(mask), dev(recs),
                                         None if upd_mask is None else dev(upd_mask), ws=ws)
    return host(d_attrs), int(host(applied)[0]), int(host(dropped)[0])


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [0.0, 0.001, 0.05, 0.5, 1.0])
@pytest.mark.parametrize("q_frac", [0.0, 0.5, 1.0, 1.5])
def test_select_update_parity(abm, orc, n, p, q_frac):
    A = 3
    attrs = W.int32_rows(n * 13 + 1, A, n)
    mask = W.bernoulli_mask(n, p, n)
    k = int(mask.sum())
    q = int(q_frac * k) if k else int(q_frac * 10)
    recs = W.int32_rows(n * 13 + 2, A, q)
    exp, ea, ed = orc.select_update(attrs, mask, recs)
    got, ga, gd = _run_select(abm, attrs, mask, recs)
    assert (ga, gd) == (ea, ed)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n,m", [(0, 0), (0, 50), (50, 0), (1000, 3000), (20000, 9000),
                                 (3 * 4096 + 5, 2 * 4096 + 9)])
@pytest.mark.parametrize("p,pu", [(0.3, 0.7), (0.9, 0.1), (1.0, 1.0)])
def test_select_update_with_update_mask(abm, orc, n, m, p, pu):
    A = 2
    attrs = W.int32_rows(n + 5, A, n)
    recs = W.int32_rows(m + 6, A, m)
    sel = W.bernoulli_mask(n + 1, p, n)
    upd = W.bernoulli_mask(m + 2, pu, m)
    exp, ea, ed = orc.select_update(attrs, sel, recs, upd_mask=upd)
    got, ga, gd = _run_select(abm, attrs, sel, recs, upd_mask=upd)
    assert (ga, gd) == (ea, ed)
    assert np.array_equal(got, exp)


def test_shared_workspace_across_calls_of_varying_size(abm, orc):
    """One workspace reused by calls whose tile counts rise and fall: stale tile
    status words of earlier launches must never be taken as current."""
    ws = abm.workspace(300_000)
    for it, n in enumerate([300_000, 5, 70_000, 4097, 300_000, 64, 123_456, 200_000]):
        A = 1 + it % 4
        attrs = W.int32_rows(it, A, n)
        mask = W.bernoulli_mask(it, 0.3, n)
        recs = W.int32_rows(it + 100, A, int(mask.sum()) // 2 + 1)
        exp, ea, ed = orc.select_update(attrs, mask, recs)
        got, ga, gd = _run_select(abm, attrs, mask, recs, ws=ws)
        assert (ga, gd) == (ea, ed), (it, n)
        assert np.array_equal(got, exp), (it, n)
    assert abm.workspace_error(ws) == 0


def test_select_update_idempotent_and_deterministic(abm):
    n, A = 50_000, 4
    attrs = W.int32_rows(1, A, n)
    mask = W.bernoulli_mask(2, 0.4, n)
    recs = W.int32_rows(3, A, int(mask.sum()))
    d = dev(attrs)
    abm.select_update(d, dev(mask), dev(recs))
    once = host(d)
    abm.select_update(d, dev(mask), dev(recs))
    assert np.array_equal(host(d), once)
    d2 = dev(attrs)
    abm.select_update(d2, dev(mask), dev(recs))
    assert np.array_equal(host(d2), once)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("p", W.DENSITIES)
def test_select_update_full_size(abm, orc, seed, p):
    """The 2^24-slot x 8-attribute microbenchmark, all slots compared."""
    case = W.select_update_case(seed, p)
    exp, ea, ed = orc.select_update(case.attrs, case.mask, case.records)
    got, ga, gd = _run_select(abm, case.attrs, case.mask, case.records)
    assert (ga, gd) == (ea, ed) == (case.k, 0)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("free_p", [0.0, 0.05, 0.5, 1.0])
@pytest.mark.parametrize("q_frac", [0.0, 0.7, 1.0, 2.0])
def test_add_agents_parity(abm, orc, n, free_p, q_frac):
    A = 2
    attrs = W.int32_rows(n + 7, A, n)
    alive = (1 - W.bernoulli_mask(n + 3, free_p, n)).astype(np.int32) * 3
    nfree = int(np.count_nonzero(alive == 0))
    q = int(q_frac * nfree) if nfree else int(q_frac * 5)
    recs = W.int32_rows(n + 8, A, q)
    exp, exp_alive, ea, ed = orc.add_agents(attrs, alive, recs)
    d_attrs, d_alive = dev(attrs), dev(alive)
    added, dropped = abm.add_agents(d_attrs, d_alive, dev(recs))
    assert (int(host(added)[0]), int(host(dropped)[0])) == (ea, ed)
    assert np.array_equal(host(d_attrs), exp)
    assert np.array_equal(host(d_alive), exp_alive)


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("p", W.DENSITIES)
def test_add_remove_full_size(abm, orc, seed, p):
    """add_agents with free density p and k newborns, then remove_agents with the
    same mask over the (now all-live) population: both at 2^24 x 8, seeds 0-9."""
    case = W.select_update_case(seed, p)
    alive = (1 - case.mask).astype(np.int32)
    exp, exp_alive, ea, ed = orc.add_agents(case.attrs, alive, case.records)
    d_attrs, d_alive = dev(case.attrs), dev(alive)
    added, dropped = abm.add_agents(d_attrs, d_alive, dev(case.records))
    assert (int(host(added)[0]), int(host(dropped)[0])) == (ea, ed) == (case.k, 0)
    assert np.array_equal(host(d_attrs), exp)
    assert np.array_equal(host(d_alive), exp_alive)
    assert np.all(exp_alive == 1)
    exp_alive2, er = orc.remove_agents(exp_alive, case.mask)
    removed = abm.remove_agents(d_alive, dev(case.mask))
    assert int(host(removed)[0]) == er == case.k
    assert np.array_equal(host(d_alive), exp_alive2)
    assert np.array_equal(exp_alive2, alive)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [0.0, 0.01, 0.5, 1.0])
def test_remove_agents_parity(abm, orc, n, p):
    alive = (1 - W.bernoulli_mask(n + 11, 0.3, n)).astype(np.int32)
    kill = W.bernoulli_mask(n + 12, p, n) * np.uint8(5)
    exp, er = orc.remove_agents(alive, kill)
    d_alive = dev(alive)
    removed = abm.remove_agents(d_alive, dev(kill))
    assert int(host(removed)[0]) == er
    assert np.array_equal(host(d_alive), exp)


def test_remove_agents_repeated_calls_share_counter(abm, orc):
    """The done/sum word re-arms itself: back-to-back calls on one workspace."""
    ws = abm.workspace(200_000)
    for it, n in enumerate([200_000, 17, 4096 * 16, 1, 150_001]):
        alive = (1 - W.bernoulli_mask(it, 0.2, n)).astype(np.int32)
        kill = W.bernoulli_mask(it + 50, 0.4, n)
        exp, er = orc.remove_agents(alive, kill)
        d_alive = dev(alive)
        removed = abm.remove_agents(d_alive, dev(kill), ws=ws)
        assert int(host(removed)[0]) == er, (it, n)
        assert np.array_equal(host(d_alive), exp)
    assert abm.workspace_error(ws) == 0


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", [0.0, 0.02, 0.5, 1.0])
def test_select_indices_parity(abm, orc, n, p):
    mask = W.bernoulli_mask(n + 21, p, n)
    exp = orc.select_indices(mask)
    out, count = abm.select_indices(dev(mask))
    k = int(host(count)[0])
    assert k == exp.size
    assert np.array_equal(host(out)[:k].astype(np.int64), exp)


@pytest.mark.parametrize("n_claims,n_targets", [(0, 0), (0, 10), (10, 0), (1, 1), (1000, 7),
                                                (50_000, 50_000), (1_000_000, 100_000)])
@pytest.mark.parametrize("with_active", [False, True])
def test_resolve_conflicts_parity(abm, orc, n_claims, n_targets, with_active):
    g = np.random.default_rng(n_claims + n_targets)
    target = g.integers(-2, n_targets + 2, size=n_claims).astype(np.int32)
    prio = g.integers(0, 8, size=n_claims).astype(np.uint32)  # many ties
    active = (g.random(n_claims) < 0.8).astype(np.uint8) if with_active else None
    eb, ew, ewon = orc.resolve_conflicts(target, prio, n_targets, active=active)
    best, winner, won = abm.resolve_conflicts(
        dev(target), dev(prio.view(np.int32)).view(torch.uint32), n_targets,
        active=None if active is None else dev(active))
    if n_targets:
        assert np.array_equal(host(best)[:n_targets], eb)
        assert np.array_equal(host(winner)[:n_targets], ew)
    if n_claims:
        assert np.array_equal(host(won)[:n_claims], ewon)


def test_resolve_conflicts_full_priority_range(abm, orc):
    g = np.random.default_rng(99)
    n, t = 3_000_000, 4_194_304
    target = g.integers(0, t, size=n).astype(np.int32)
    prio = g.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    eb, ew, ewon = orc.resolve_conflicts(target, prio, t)
    best, winner, won = abm.resolve_conflicts(dev(target),
                                              dev(prio.view(np.int32)).view(torch.uint32), t)
    assert np.array_equal(host(best), eb)
    assert np.array_equal(host(winner), ew)
    assert np.array_equal(host(won), ewon)


def test_graph_replay_select_add_remove(abm, orc):
    """select_update, add_agents and remove_agents recorded once into a graph and
    replayed with fresh inputs copied in between: the device-side epoch keeps
    every replay's scan separate from the last one's."""
    n, A, k = 200_000, 4, 30_000
    ws = abm.workspace(n)
    cnt = torch.zeros(8, dtype=torch.int64, device="cuda")
    d_attrs = torch.zeros((A, n), dtype=torch.int32, device="cuda")
    d_mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
    d_recs = torch.zeros((A, k), dtype=torch.int32, device="cuda")
    d_alive = torch.ones(n, dtype=torch.int32, device="cuda")
    d_kill = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        # warm-up outside capture (library load, device check)
        abm.select_update(d_attrs, d_mask, d_recs, ws=ws, applied=cnt[0:1], dropped=cnt[1:2])
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        abm.select_update(d_attrs, d_mask, d_recs, ws=ws, applied=cnt[0:1], dropped=cnt[1:2])
        abm.add_agents(d_attrs, d_alive, d_recs, ws=ws, added=cnt[2:3], dropped=cnt[3:4])
        abm.remove_agents(d_alive, d_kill, ws=ws, removed=cnt[4:5])
    for it in range(6):
        attrs = W.int32_rows(100 + it, A, n)
        mask = W.bernoulli_mask(200 + it, 0.1 + 0.1 * it, n)
        recs = W.int32_rows(300 + it, A, k)
        alive = (1 - W.bernoulli_mask(400 + it, 0.2, n)).astype(np.int32)
        kill = W.bernoulli_mask(500 + it, 0.3, n)
        d_attrs.copy_(dev(attrs))
        d_mask.copy_(dev(mask))
        d_recs.copy_(dev(recs))
        d_alive.copy_(dev(alive))
        d_kill.copy_(dev(kill))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e1, ea, ed = orc.select_update(attrs, mask, recs)
        e2, eal, eadd, edrop = orc.add_agents(e1, alive, recs)
        eal2, erem = orc.remove_agents(eal, kill)
        c = host(cnt)
        assert (c[0], c[1], c[2], c[3], c[4]) == (ea, ed, eadd, edrop, erem), it
        assert np.array_equal(host(d_attrs), e2), it
        assert np.array_equal(host(d_alive), eal2), it
    assert abm.workspace_error(ws) == 0
