"""GPU parity of the predation model (Sec. 5.1) against the CPU oracle.

Bit-exact comparison of every state array (grass countdowns; x, y, energy and
alive of both species, including stale fields of free slots) and of the
per-step statistics.  The small 64x64 workload is compared after every one of
its 200 steps for seeds 0-9; tiny tori put every agent in conflict; the large
2048x2048 workload (16M / 4M slots) is compared in full after each of its
first steps and after step 100 (with the statistics of every step up to it),
and checked through population bookkeeping for all 1000 steps.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "e", "alive")


def _host(t):
    return t.cpu().numpy()


def _assert_same(model, S, where=""):
    torch.cuda.synchronize()
    assert np.array_equal(_host(model.grass), S.grass), f"grass {where}"
    for sp in ("sheep", "wolves"):
        g = getattr(model, sp)
        o = getattr(S, sp)
        for f in FIELDS:
            a, b = _host(g[f]), o[f]
            if not np.array_equal(a, b):
                bad = np.flatnonzero(a != b)
                raise AssertionError(f"{sp}.{f} {where}: {bad.size} slots differ, first "
                                     f"{bad[:5]} gpu {a[bad[:5]]} oracle {b[bad[:5]]}")


def _pair(abm, orc, **kw):
    P = orc.pred_params(**kw)
    S = orc.predation_init(P)
    model = abm.predation_init(abm.predation_params(**kw))
    return P, S, model


@pytest.mark.parametrize("seed", range(10))
def test_small_workload_every_step(abm, orc, seed):
    """64x64, 400 sheep / 100 wolves in 4096 / 1024 slots, 200 steps."""
    P, S, model = _pair(abm, orc, seed=seed)
    _assert_same(model, S, "after init")
    stats = torch.zeros((1, 8), dtype=torch.int64, device="cuda")
    for t in range(200):
        exp = orc.predation_step(P, S)
        model.run(1, stats)
        got = dict(zip(abm.STAT_NAMES, (int(v) for v in _host(stats)[0])))
        assert got == exp, f"stats step {t}"
        _assert_same(model, S, f"after step {t}")
    assert abm.workspace_error(model.ws) == 0


@pytest.mark.parametrize("W,H,cap_s,cap_w,n_s0,n_w0", [
    (1, 1, 6, 4, 3, 2), (2, 1, 6, 4, 4, 2), (3, 3, 8, 6, 5, 3), (5, 3, 40, 9, 20, 6),
    (17, 9, 5000, 3000, 900, 400),
])
def test_tiny_tori_many_seeds(abm, orc, W, H, cap_s, cap_w, n_s0, n_w0):
    """All agents share few cells, so every conflict outcome occurs; capacities
    overflow; multi-tile species on the last case."""
    for seed in range(12):
        kw = dict(W=W, H=H, R=3, T_s=2 ** 31, T_w=2 ** 31, seed=seed, cap_s=cap_s, cap_w=cap_w,
                  n_s0=n_s0, n_w0=n_w0)
        P, S, model = _pair(abm, orc, **kw)
        for t in range(15):
            orc.predation_step(P, S)
            model.run(1)
            _assert_same(model, S, f"seed {seed} step {t}")


def test_multi_step_call_matches_single_steps(abm, orc):
    """One call of 200 steps = 200 calls of one step; stats rows line up."""
    P, S, model = _pair(abm, orc, seed=5)
    stats = torch.zeros((200, 8), dtype=torch.int64, device="cuda")
    model.run(200, stats)
    exp = orc.predation_run(P, S, 200)
    assert model.step == S.step == 200
    got = _host(stats)
    for t in range(200):
        assert dict(zip(abm.STAT_NAMES, (int(v) for v in got[t]))) == exp[t], t
    _assert_same(model, S, "after 200 steps")


def test_resume_from_copied_state(abm, orc):
    """Draws are keyed on (seed, step): a copy of the state resumed on a fresh
    model continues bit-exactly."""
    P, S, model = _pair(abm, orc, seed=8)
    model.run(40)
    clone = abm.PredationModel.create(model.params)
    clone.grass.copy_(model.grass)
    for sp in ("sheep", "wolves"):
        for f in FIELDS:
            getattr(clone, sp)[f].copy_(getattr(model, sp)[f])
    clone.step = model.step
    clone.run(40)
    orc.predation_run(P, S, 80)
    _assert_same(clone, S, "resumed")


def test_large_workload(abm, orc):
    """2048x2048, capacities 2^24 sheep / 2^22 wolves, 1.6M / 0.4M initial."""
    kw = dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000, n_w0=400_000,
              seed=0)
    P, S, model = _pair(abm, orc, **kw)
    _assert_same(model, S, "after init")
    for t in range(3):
        orc.predation_step(P, S)
        model.run(1)
        _assert_same(model, S, f"after step {t}")
    # the rest of the 1000 steps: population bookkeeping from the device stats
    n = 997
    stats = torch.zeros((n, 8), dtype=torch.int64, device="cuda")
    model.run(n, stats)
    st = _host(stats)
    for t in range(n - 1):
        live_s, live_w, ge, se, bs, bw, ss, sw = (int(v) for v in st[t])
        assert st[t + 1][0] == live_s - se - ss + bs, t
        assert st[t + 1][1] == live_w - sw + bw, t
        assert 0 <= bs <= P.cap_s - (live_s - se) and 0 <= bw <= P.cap_w - live_w
        assert ge <= P.W * P.H and se <= live_s
    alive_s = int(_host(model.sheep["alive"]).sum())
    assert alive_s == st[n - 1][0] - st[n - 1][3] - st[n - 1][6] + st[n - 1][4]
    assert abm.workspace_error(model.ws) == 0


def test_large_workload_full_state_at_step_100(abm, orc):
    """2048x2048 as above: the statistics of each of the first 100 steps and the
    whole state (4M grass cells, 16M + 4M slots) after step 100."""
    kw = dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000, n_w0=400_000,
              seed=1)
    P, S, model = _pair(abm, orc, **kw)
    n = 100
    stats = torch.zeros((n, 8), dtype=torch.int64, device="cuda")
    model.run(n, stats)
    exp = orc.predation_run(P, S, n)
    got = _host(stats)
    for t in range(n):
        assert dict(zip(abm.STAT_NAMES, (int(v) for v in got[t]))) == exp[t], f"stats step {t}"
    _assert_same(model, S, f"after step {n}")
    assert abm.workspace_error(model.ws) == 0


# ---------------------------------------------------------------- multi-prey
@pytest.mark.parametrize("seed", range(4))
def test_multi_prey_small_workload_every_step(abm, orc, seed):
    """multi_prey = 1 on the 64x64 workload: state and statistics after every
    one of 200 steps."""
    P, S, model = _pair(abm, orc, seed=seed, multi_prey=1)
    stats = torch.zeros((1, 8), dtype=torch.int64, device="cuda")
    for t in range(200):
        exp = orc.predation_step(P, S)
        model.run(1, stats)
        got = dict(zip(abm.STAT_NAMES, (int(v) for v in _host(stats)[0])))
        assert got == exp, f"stats step {t}"
        _assert_same(model, S, f"after step {t}")


@pytest.mark.parametrize("W,H,cap_s,cap_w,n_s0,n_w0", [
    (1, 1, 40, 20, 12, 6), (2, 1, 30, 30, 14, 14), (3, 3, 60, 40, 30, 25), (17, 9, 5000, 3000, 900, 400),
])
def test_multi_prey_crowded_cells(abm, orc, W, H, cap_s, cap_w, n_s0, n_w0):
    """Tens of wolves and sheep on one cell: every rank of the per-cell
    matching is exercised, with more sheep than wolves and the reverse."""
    for seed in range(8):
        kw = dict(W=W, H=H, R=3, T_s=2 ** 30, T_w=2 ** 30, seed=seed, cap_s=cap_s, cap_w=cap_w,
                  n_s0=n_s0, n_w0=n_w0, multi_prey=1)
        P, S, model = _pair(abm, orc, **kw)
        stats = torch.zeros((1, 8), dtype=torch.int64, device="cuda")
        for t in range(12):
            exp = orc.predation_step(P, S)
            model.run(1, stats)
            assert dict(zip(abm.STAT_NAMES, (int(v) for v in _host(stats)[0]))) == exp
            _assert_same(model, S, f"seed {seed} step {t}")


def test_multi_prey_large_workload(abm, orc):
    """2048x2048 with multi_prey: two full comparisons, then bookkeeping."""
    kw = dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000, n_w0=400_000,
              seed=2, multi_prey=1)
    P, S, model = _pair(abm, orc, **kw)
    for t in range(2):
        orc.predation_step(P, S)
        model.run(1)
        _assert_same(model, S, f"after step {t}")
    n = 100
    stats = torch.zeros((n, 8), dtype=torch.int64, device="cuda")
    model.run(n, stats)
    st = _host(stats)
    for t in range(n - 1):
        live_s, live_w, ge, se, bs, bw, ss, sw = (int(v) for v in st[t])
        assert st[t + 1][0] == live_s - se - ss + bs, t
        assert st[t + 1][1] == live_w - sw + bw, t
        assert se <= min(live_s, live_w)
    assert abm.workspace_error(model.ws) == 0
