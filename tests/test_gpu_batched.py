"""GPU parity of the batched predation form (many uneven models, one launch).

Each model of a batch must be bit-identical to the same model run alone by the
oracle: grass countdowns, every species array (stale fields included), the
step counter, the live counts and the agent-update count (live agents at the
start of each step, summed).
"""
import numpy as np
import pytest
import torch

from paper_2508_16508_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "e", "alive")


def _host(t):
    return t.cpu().numpy()


def _params(abm, orc, **kw):
    return abm.predation_params(**kw), orc.pred_params(**kw)


def _check_model(abm, orc, batch, m, kw, steps, countdown):
    P = orc.pred_params(**kw)
    S = orc.predation_init(P)
    st = orc.predation_run(P, S, steps)
    grass, sheep, wolves = batch.model_state(m, countdown)
    assert np.array_equal(_host(grass), S.grass), (m, "grass")
    for name, g, o in (("sheep", sheep, S.sheep), ("wolves", wolves, S.wolves)):
        for f in FIELDS:
            a, b = _host(g[f]), o[f]
            if not np.array_equal(a, b):
                bad = np.flatnonzero(a != b)
                raise AssertionError(f"model {m} {name}.{f}: {bad.size} differ, first {bad[:5]} "
                                     f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    d = batch.descriptors()[m]
    assert d.step == steps
    assert d.updates == sum(s["live_s"] + s["live_w"] for s in st)
    assert d.live_s == int(np.count_nonzero(S.sheep["alive"]))
    assert d.live_w == int(np.count_nonzero(S.wolves["alive"]))


def _mixed_models(seed, n):
    g = np.random.default_rng(seed)
    out = []
    for m in range(n):
        Wd = int(g.integers(1, 41))
        Hd = int(g.integers(1, 41))
        cells = Wd * Hd
        cap_s = int(g.integers(1, max(2, cells // 2) + 1))
        cap_w = int(g.integers(1, max(2, cells // 6) + 1))
        kw = dict(W=Wd, H=Hd, R=int(g.integers(1, 12)), seed=int(g.integers(0, 2 ** 32)),
                  cap_s=cap_s, cap_w=cap_w, n_s0=int(g.integers(0, cap_s + 1)),
                  n_w0=int(g.integers(0, cap_w + 1)), T_s=int(g.integers(0, 2 ** 31)),
                  T_w=int(g.integers(0, 2 ** 31)))
        out.append(kw)
    return out


@pytest.mark.parametrize("block,items", [(256, 1), (512, 2), (512, 4), (1024, 2)])
def test_mixed_batch_matches_models_alone(abm, orc, block, items):
    """40 models of random shapes (1x1 up to 40x40, tiny and overflowing
    capacities, different regrowth delays, seeds and reproduction rates),
    different step targets, advanced in three launches of at most 12 steps."""
    kws = _mixed_models(block + items, 40)
    targets = [int(t) for t in np.random.default_rng(7).integers(0, 31, size=len(kws))]
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], targets,
                                 block_threads=block, items=items)
    batch.init()
    for _ in range(3):
        batch.run(12)
    torch.cuda.synchronize()
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, min(targets[m], 36), cd)


def test_small_workload_in_a_batch(abm, orc):
    """The 64x64 model (seeds 0-7) inside a batch for all 200 steps."""
    kws = [dict(seed=s) for s in range(8)]
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 200)
    batch.init()
    batch.run(200)
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, 200, cd)


def test_uneven_workload_sample(abm, orc):
    """Models of the 4096-model workload recipe (side 32-256, sheep = cells/10,
    wolves = cells/40, capacities 4x): the smallest, the largest and a spread
    between, 60 steps."""
    specs = W.batched_models(0, 4096)
    by_side = sorted(range(len(specs)), key=lambda m: specs[m].side)
    pick = [by_side[i] for i in (0, 1, 500, 1500, 2500, 3500, 4094, 4095)]
    kws = []
    for m in pick:
        sp = specs[m]
        kws.append(dict(W=sp.side, H=sp.side, seed=sp.seed, cap_s=sp.cap_s, cap_w=sp.cap_w,
                        n_s0=sp.n_s0, n_w0=sp.n_w0))
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 60)
    batch.init()
    batch.run(25)
    batch.run(35)
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, 60, cd)


def test_batched_equals_one_model_path(abm):
    """The same model advanced by the batched launch and by the one-model
    multi-launch path ends in identical bytes."""
    kw = dict(W=96, H=80, seed=33, cap_s=3000, cap_w=800, n_s0=700, n_w0=200)
    batch = abm.BatchedPredation([abm.predation_params(**kw)] * 3, [50, 50, 20])
    batch.init()
    batch.run(50)
    plain = abm.predation_init(abm.predation_params(**kw))
    plain.run(50)
    grass, sheep, wolves = batch.model_state(1)
    assert torch.equal(grass, plain.grass)
    for f in FIELDS:
        assert torch.equal(sheep[f], plain.sheep[f]) and torch.equal(wolves[f], plain.wolves[f])
    d = batch.descriptors()
    assert (d[0].step, d[1].step, d[2].step) == (50, 50, 20)


def test_autotuner_picks_a_candidate_and_caches_it(abm, tmp_path):
    from paper_2508_16508_amd.tune import autotune_batched
    kws = [dict(W=40 + m, H=30, seed=m, cap_s=900, cap_w=200, n_s0=120, n_w0=30)
           for m in range(16)]

    def make(block, items):
        b = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 100,
                                 block_threads=block, items=items)
        b.init()
        return b

    path = str(tmp_path / "tune.json")
    cands = ((256, 2), (512, 4))
    first = autotune_batched(make, "test", steps=3, candidates=cands, cache_path=path)
    assert not first["cached"] and (first["block_threads"], first["items"]) in cands
    assert set(first["timings_ms"]) == {"256x2", "512x4"}
    again = autotune_batched(make, "test", steps=3, candidates=cands, cache_path=path)
    assert again["cached"] and again["block_threads"] == first["block_threads"]


def _team_models(seed):
    """Big models (split over a team) and small ones (one workgroup each):
    capacities below, at and above the team size, a species with no agents,
    a species larger than the grid, a 1-row torus."""
    g = np.random.default_rng(seed)
    kws = [dict(W=120, H=100, seed=int(g.integers(0, 2 ** 32)), cap_s=4800, cap_w=1200,
                n_s0=1200, n_w0=300),
           dict(W=200, H=90, seed=int(g.integers(0, 2 ** 32)), cap_s=20000, cap_w=3, n_s0=1800,
                n_w0=3, T_w=2 ** 31 - 1),
           dict(W=150, H=1, seed=int(g.integers(0, 2 ** 32)), cap_s=7000, cap_w=7000, n_s0=15,
                n_w0=4, R=3),
           dict(W=110, H=110, seed=int(g.integers(0, 2 ** 32)), cap_s=5000, cap_w=1, n_s0=900,
                n_w0=0),
           dict(W=100, H=100, seed=int(g.integers(0, 2 ** 32)), cap_s=12000, cap_w=2500,
                n_s0=3000, n_w0=800, T_s=2 ** 30, T_w=2 ** 30)]
    kws += _mixed_models(seed + 1, 12)
    return kws


@pytest.mark.parametrize("K,block,items", [(2, 256, 1), (4, 512, 4), (8, 256, 2), (16, 512, 4)])
def test_teams_match_models_alone(abm, orc, K, block, items):
    """Models of at least 6000 cells plus slots are advanced by teams of K
    workgroups (three team barriers per step), the rest by one workgroup; every
    model must match the oracle run alone, over three launches."""
    kws = _team_models(K)
    targets = [40, 33, 40, 12, 40] + [int(t) for t in np.random.default_rng(K).integers(0, 41, 12)]
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], targets,
                                 block_threads=block, items=items, team_size=K,
                                 team_min_size=6000)
    assert batch.team_models() == 5
    batch.init()
    for _ in range(3):
        batch.run(14)
    torch.cuda.synchronize()
    assert abm.workspace_error(batch.ws) == 0
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, min(targets[m], 42), cd)


def test_team_equals_one_workgroup_on_a_large_model(abm):
    """A 1024x1024 model of the served-trace recipe (sheep = cells/10, wolves =
    cells/40, capacities 4x), 30 steps by a team of 16 and by one workgroup:
    identical bytes."""
    L = 1024
    kw = dict(W=L, H=L, seed=77, cap_s=4 * (L * L // 10), cap_w=4 * (L * L // 40),
              n_s0=L * L // 10, n_w0=L * L // 40)
    out = []
    for k in (16, 1):
        b = abm.BatchedPredation([abm.predation_params(**kw)], 30, team_size=k, team_min_size=1)
        b.init()
        b.run(30)
        torch.cuda.synchronize()
        assert abm.workspace_error(b.ws) == 0
        out.append((b.grass_countdown(), b.sheep, b.wolves, b.descriptors()[0]))
    (g0, s0, w0, d0), (g1, s1, w1, d1) = out
    assert torch.equal(g0, g1)
    for f in FIELDS:
        assert torch.equal(s0[f], s1[f]) and torch.equal(w0[f], w1[f])
    assert (d0.step, d0.updates, d0.live_s, d0.live_w) == (d1.step, d1.updates, d1.live_s,
                                                           d1.live_w)


def test_team_launch_rejects_bad_tuning(abm):
    kw = dict(W=64, H=64, seed=1)
    b = abm.BatchedPredation([abm.predation_params(**kw)] * 2, 5, team_size=2, team_min_size=1)
    b.init()
    with pytest.raises(abm.AbmError, match="team_size"):
        b.run(5, team_size=17)
    with pytest.raises(abm.AbmError, match="resident"):
        b.run(5, workgroups=15)                      # teams of 2 need 16 workgroups
    with pytest.raises(abm.AbmError, match="multiple"):
        b.run(5, team_workgroups=24)
    b.run(5, workgroups=16)
    d = b.descriptors()
    assert d[0].step == 5 and d[1].step == 5


@pytest.mark.parametrize("team_size", [1, 2])
def test_resume_from_an_edited_state(abm, orc, team_size):
    """Between launches, agents are killed in low slots and placed in the
    highest slots: the next launch scans every slot of each species, finds
    every live agent wherever it sits, and matches the oracle run from the
    edited state."""
    kws = [dict(W=48, H=40, seed=3, cap_s=3000, cap_w=900, n_s0=300, n_w0=80),
           dict(W=30, H=30, seed=9, cap_s=1000, cap_w=400, n_s0=100, n_w0=30)]
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 40,
                                 team_size=team_size, team_min_size=1)
    batch.init()
    batch.run(10)
    g = np.random.default_rng(team_size)
    cd = batch.grass_countdown()
    starts = []
    for m, kw in enumerate(kws):
        grass, sheep, wolves = batch.model_state(m, cd)
        host = {}
        for name, sp, cap in (("sheep", sheep, kw["cap_s"]), ("wolves", wolves, kw["cap_w"])):
            arr = {f: _host(sp[f]).copy() for f in FIELDS}
            live = np.flatnonzero(arr["alive"])
            arr["alive"][live[g.random(live.size) < 0.3]] = 0
            top = np.arange(cap - 5, cap)
            arr["alive"][top] = 1
            arr["x"][top] = g.integers(0, kw["W"], 5)
            arr["y"][top] = g.integers(0, kw["H"], 5)
            arr["e"][top] = g.integers(1, 20, 5)
            for f in FIELDS:
                sp[f].copy_(torch.from_numpy(arr[f]))
            host[name] = arr
        starts.append(orc.PredState(_host(grass).copy(), host["sheep"], host["wolves"], 10))
    torch.cuda.synchronize()
    batch.run(30)
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        S = starts[m]
        orc.predation_run(orc.pred_params(**kw), S, 30)
        grass, sheep, wolves = batch.model_state(m, cd)
        assert np.array_equal(_host(grass), S.grass), m
        for name, gsp, osp in (("sheep", sheep, S.sheep), ("wolves", wolves, S.wolves)):
            for f in FIELDS:
                assert np.array_equal(_host(gsp[f]), osp[f]), (m, name, f)
        assert batch.descriptors()[m].step == 40


def test_captured_rollout_replays_match_oracle(abm, orc):
    """A rollout captured by the library (three launches of 10 steps) replayed
    twice, with eager device work and synchronisation between the replays: the
    state after each replay matches the oracle after 30 and 60 steps."""
    kws = [dict(W=40, H=40, seed=21, cap_s=640, cap_w=160, n_s0=160, n_w0=40),
           dict(W=25, H=31, seed=22, cap_s=300, cap_w=80, n_s0=77, n_w0=19),
           dict(W=64, H=64, seed=23, cap_s=4096, cap_w=1024, n_s0=400, n_w0=100)]
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 60)
    batch.init()
    graph = batch.capture(10, 3)
    torch.cuda.synchronize()
    assert all(d.step == 0 for d in batch.descriptors())     # capture runs nothing
    for steps in (30, 60):
        graph.replay()
        torch.cuda.synchronize()
        checksum = int(batch.sheep["e"].to(torch.int64).sum().item())   # eager work between
        cd = batch.grass_countdown()
        for m, kw in enumerate(kws):
            _check_model(abm, orc, batch, m, kw, steps, cd)
        assert checksum == int(batch.sheep["e"].to(torch.int64).sum().item())
    graph.replay()                                           # every model is at its target
    torch.cuda.synchronize()
    assert all(d.step == 60 for d in batch.descriptors())
    graph.destroy()
    assert abm.workspace_error(batch.ws) == 0


def test_full_workload_graph_replay(abm, orc):
    """The 4096-model workload (side 32-256) as the benchmark runs it: one
    warm-up step, then 499 steps replayed from a library-captured graph of
    50-step persistent launches.  Every model's whole state and counters
    equal those of the same batch advanced without a graph, with another
    launch shape (1024 x 4, teams of 4 for the 64 largest models, 100-step
    launches, every claim table global, where the benchmark keeps the
    smallest models' tables in LDS); 48 models across the sizes equal the
    one-model multi-launch path; 12 of them equal the oracle."""
    specs = W.batched_models(0, 4096)
    kws = [dict(W=sp.side, H=sp.side, seed=sp.seed, cap_s=sp.cap_s, cap_w=sp.cap_w,
                n_s0=sp.n_s0, n_w0=sp.n_w0) for sp in specs]
    params = [abm.predation_params(**kw) for kw in kws]
    steps = 500
    a = abm.BatchedPredation(params, steps, block_threads=512, items=2)
    a.init()
    a.run(1)
    graph = a.capture(50, 10)
    graph.replay()
    assert a.lds_models() > 0
    b = abm.BatchedPredation(params, steps, block_threads=1024, items=4, team_size=4,
                             team_min_size=a.sorted_size[63], lds=False)
    b.init()
    for _ in range(5):
        b.run(100)
    torch.cuda.synchronize()
    assert abm.workspace_error(a.ws) == 0 and abm.workspace_error(b.ws) == 0
    da, db = a.descriptors(), b.descriptors()
    assert all(d.step == steps for d in da)
    for m in range(len(specs)):
        assert (da[m].updates, da[m].live_s, da[m].live_w) == \
            (db[m].updates, db[m].live_s, db[m].live_w), m
    ca, cb = a.grass_countdown(), b.grass_countdown()
    assert torch.equal(ca, cb)
    for f in FIELDS:
        assert torch.equal(a.sheep[f], b.sheep[f]) and torch.equal(a.wolves[f], b.wolves[f]), f
    del b, cb
    torch.cuda.empty_cache()
    by_side = sorted(range(len(specs)), key=lambda m: specs[m].side)
    pick = [by_side[i] for i in np.linspace(0, len(specs) - 1, 48).astype(int)]
    for m in pick:
        plain = abm.predation_init(params[m])
        plain.run(steps)
        grass, sheep, wolves = a.model_state(m, ca)
        assert torch.equal(grass, plain.grass), m
        for f in FIELDS:
            assert torch.equal(sheep[f], plain.sheep[f]) and torch.equal(wolves[f],
                                                                          plain.wolves[f]), (m, f)
    for m in pick[::4]:
        _check_model(abm, orc, a, m, kws[m], steps, ca)
    graph.destroy()


def test_lds_claim_tables_match_global_ones(abm, orc):
    """Models on both sides of the LDS limit of each launch shape (claim tables
    of 24 bytes per cell) run with claims in LDS where they fit and with every
    claim table global: identical bytes, the global claim table all-ones after
    every run, and models on both sides of the limit match the oracle."""
    props = torch.cuda.get_device_properties(0)
    for block, items in ((512, 2), (1024, 4), (256, 1)):
        lim = int(abm.lib().abm_batched_lds_cells(block, items))
        assert 1024 <= lim and 24 * lim <= getattr(props, "shared_memory_per_block", 24 * lim)
        side = int(np.sqrt(lim))
        g = np.random.default_rng(block + items)
        kws = []
        for (Wd, Hd) in ((side, side), (side + 1, side + 1), (lim, 1), (1, lim + 1), (3, 5),
                         (side + 20, side), (17, 40)):
            cells = Wd * Hd
            kws.append(dict(W=Wd, H=Hd, seed=int(g.integers(0, 2 ** 32)), cap_s=cells // 2 + 1,
                            cap_w=cells // 8 + 1, n_s0=cells // 10, n_w0=cells // 40 + 1,
                            R=int(g.integers(1, 12))))
        params = [abm.predation_params(**kw) for kw in kws]
        out = []
        for lds in (True, False):
            b = abm.BatchedPredation(params, 45, block_threads=block, items=items, lds=lds)
            assert b.lds_models() == (4 if lds else 0)
            b.init()
            for steps in (20, 25):
                b.run(steps)
            torch.cuda.synchronize()
            assert abm.workspace_error(b.ws) == 0
            assert bool((b.claims.view(torch.int64) == -1).all()), lds
            out.append(b)
        cds = [b.grass_countdown() for b in out]
        assert torch.equal(cds[0], cds[1])
        for f in FIELDS:
            assert torch.equal(out[0].sheep[f], out[1].sheep[f])
            assert torch.equal(out[0].wolves[f], out[1].wolves[f])
        for d0, d1 in zip(out[0].descriptors(), out[1].descriptors()):
            assert (d0.step, d0.updates, d0.live_s, d0.live_w) == \
                (d1.step, d1.updates, d1.live_s, d1.live_w)
        for m in (0, 1, 4):
            _check_model(abm, orc, out[0], m, kws[m], 45, cds[0])
        del out, cds
        torch.cuda.empty_cache()


def test_lds_cells_rejects_bad_shapes(abm):
    assert abm.lib().abm_batched_lds_cells(100, 2) == 0
    assert abm.lib().abm_batched_lds_cells(512, 8) == 0
    # fewer workgroups resident per CU leave each more LDS
    assert abm.lib().abm_batched_lds_cells(1024, 1) >= abm.lib().abm_batched_lds_cells(256, 1)


def _multi_models(seed):
    """Crowded multi-prey tori (tens of each species on one cell, more sheep
    than wolves and the reverse), the 64x64 workload with multi-prey, and
    one-prey models beside them."""
    g = np.random.default_rng(seed)
    kws = []
    for (Wd, Hd, cs, cw, ns, nw) in ((1, 1, 40, 20, 12, 6), (2, 1, 30, 30, 14, 14),
                                     (3, 3, 60, 40, 30, 25), (17, 9, 5000, 3000, 900, 400),
                                     (1, 1, 25, 60, 5, 30)):
        kws.append(dict(W=Wd, H=Hd, R=3, T_s=2 ** 30, T_w=2 ** 30,
                        seed=int(g.integers(0, 2 ** 32)), cap_s=cs, cap_w=cw, n_s0=ns, n_w0=nw,
                        multi_prey=1))
    kws.append(dict(seed=int(g.integers(0, 2 ** 32)), multi_prey=1))
    kws.append(dict(W=150, H=120, seed=int(g.integers(0, 2 ** 32)), cap_s=9000, cap_w=3000,
                    n_s0=3000, n_w0=1500, multi_prey=1))
    kws += _mixed_models(seed + 3, 6)
    return kws


@pytest.mark.parametrize("block,items,lds", [(512, 2, True), (256, 1, False), (1024, 4, True)])
def test_multi_prey_models_in_a_batch(abm, orc, block, items, lds):
    """Multi-prey models (prey matched by rank within each cell) beside
    one-prey models in one batch, claims in LDS where they fit or all global,
    over two launches: every model matches the oracle run alone, and the
    global claim table (list heads included) is all-ones afterwards."""
    kws = _multi_models(block + items)
    targets = [24, 24, 24, 24, 24, 60, 30] + [20] * 6
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], targets,
                                 block_threads=block, items=items, lds=lds)
    assert batch.links is not None
    batch.init()
    batch.run(11)
    batch.run(60)
    torch.cuda.synchronize()
    assert abm.workspace_error(batch.ws) == 0
    assert bool((batch.claims.view(torch.int64) == -1).all())
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, targets[m], cd)


@pytest.mark.parametrize("K", [2, 4])
def test_multi_prey_teams_match_models_alone(abm, orc, K):
    """Multi-prey models large enough for teams (the lists of a cell hold
    agents of several members): every model matches the oracle."""
    g = np.random.default_rng(K)
    kws = [dict(W=120, H=100, seed=int(g.integers(0, 2 ** 32)), cap_s=9600, cap_w=4800,
                n_s0=4000, n_w0=2400, multi_prey=1),
           dict(W=40, H=30, seed=int(g.integers(0, 2 ** 32)), cap_s=20000, cap_w=9000,
                n_s0=6000, n_w0=3000, multi_prey=1, T_s=2 ** 30, T_w=2 ** 30),
           dict(W=100, H=100, seed=int(g.integers(0, 2 ** 32)), cap_s=12000, cap_w=2500,
                n_s0=3000, n_w0=800)]
    kws += _mixed_models(K + 10, 5)
    batch = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 30, team_size=K,
                                 team_min_size=6000)
    assert batch.team_models() == 3
    batch.init()
    batch.run(13)
    batch.run(17)
    torch.cuda.synchronize()
    assert abm.workspace_error(batch.ws) == 0
    cd = batch.grass_countdown()
    for m, kw in enumerate(kws):
        _check_model(abm, orc, batch, m, kw, 30, cd)


def test_multi_prey_batched_equals_one_model_path(abm):
    """A 512x512 multi-prey model at the workload's densities, advanced 40
    steps by a team of 8 and alone on the one-model path: identical bytes."""
    L = 512
    kw = dict(W=L, H=L, seed=91, cap_s=4 * (L * L // 10), cap_w=4 * (L * L // 40),
              n_s0=L * L // 10, n_w0=L * L // 40, multi_prey=1)
    b = abm.BatchedPredation([abm.predation_params(**kw)], 40, team_size=8, team_min_size=1)
    b.init()
    b.run(40)
    plain = abm.predation_init(abm.predation_params(**kw))
    plain.run(40)
    torch.cuda.synchronize()
    assert abm.workspace_error(b.ws) == 0
    grass, sheep, wolves = b.model_state(0)
    assert torch.equal(grass, plain.grass)
    for f in FIELDS:
        assert torch.equal(sheep[f], plain.sheep[f]) and torch.equal(wolves[f], plain.wolves[f])


def test_multi_prey_model_without_links_is_left_untouched(abm):
    kws = [dict(W=20, H=20, seed=1, multi_prey=1, cap_s=400, cap_w=100, n_s0=40, n_w0=10),
           dict(W=20, H=20, seed=2, cap_s=400, cap_w=100, n_s0=40, n_w0=10)]
    b = abm.BatchedPredation([abm.predation_params(**kw) for kw in kws], 5)
    b.init()
    b.links = None                    # the batch now passes no links
    b.run(5)
    torch.cuda.synchronize()
    d = b.descriptors()
    assert abm.workspace_error(b.ws) == 1
    assert (d[0].step, d[1].step) == (0, 5)
