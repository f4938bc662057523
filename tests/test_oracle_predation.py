"""Pins for the oracle's predation model (Sec. 5.1, Fig. 2).

The paper prints no trajectories, so the model is pinned by (i) steps worked by
hand on 1x1 and 3x3 tori, (ii) invariants checked phase by phase over many
seeds, including a brute-force per-cell search for every conflict winner, and
(iii) special cases (starvation, regrowth timing, capacity overflow).
"""
import numpy as np
import pytest

from conftest import golden_path

SPECIES = ("sheep", "wolves")
FIELDS = ("x", "y", "e", "alive")


def _load_hand(name):
    meta, exp = {}, {}
    for line in open(golden_path(name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        key, val = line.split(":", 1)
        if key == "params":
            meta = {k: int(v) for k, v in (t.split("=") for t in val.split())}
        elif key.startswith("stats."):
            exp[key] = {k: int(v) for k, v in (t.split("=") for t in val.split())}
        else:
            exp[key] = [int(v) for v in val.split()]
    return meta, exp


def _get(S, path):
    parts = path.split(".")
    if parts[-1] == "grass":
        return list(S.grass)
    return list(getattr(S, parts[-2])[parts[-1]])


@pytest.mark.parametrize("name", ["predation_hand_1x1.txt", "predation_hand_3x3.txt"])
def test_hand_worked_steps(orc, name):
    meta, exp = _load_hand(name)
    P = orc.pred_params(**meta)
    S = orc.predation_init(P)
    checked = 0
    for key, val in exp.items():
        if key.startswith("init."):
            assert _get(S, key) == val, key
            checked += 1
    for t in range(2):
        st = orc.predation_step(P, S)
        assert st == exp[f"stats.{t}"], t
        for key, val in exp.items():
            if key.startswith(f"after.{t}."):
                assert _get(S, key) == val, key
                checked += 1
    assert checked >= 12


def _cell(P, x, y):
    return np.asarray(y, dtype=np.int64) * P.W + np.asarray(x, dtype=np.int64)


def _key(orc, P, t, i, purpose):
    return (orc.rng(P.seed, t, i, purpose) << 32) | i


def _check_move(orc, P, before, after, t):
    for sp, purpose in (("sheep", 0x13), ("wolves", 0x23)):
        b, a = getattr(before, sp), getattr(after, sp)
        live = b["alive"] != 0
        assert np.array_equal(a["alive"], b["alive"])
        for f in FIELDS:
            assert np.array_equal(a[f][~live], b[f][~live])
        assert np.array_equal(a["e"][live], b["e"][live] - 1)
        dx = (a["x"][live] - b["x"][live]) % P.W
        dy = (a["y"][live] - b["y"][live]) % P.H
        # the step is one of the eight toroidal neighbours (never a stay when W, H >= 3)
        ok_x = np.isin(dx, [0, 1, P.W - 1])
        ok_y = np.isin(dy, [0, 1, P.H - 1])
        assert ok_x.all() and ok_y.all()
        if P.W >= 3 and P.H >= 3:
            assert not np.any((dx == 0) & (dy == 0))


def _check_eat(orc, P, before, after, t, ng, ns):
    """Brute-force per-cell search for grass and prey winners."""
    G = P.W * P.H
    sb, sa = before.sheep, after.sheep
    wb, wa = before.wolves, after.wolves
    live_s = np.flatnonzero(sb["alive"])
    live_w = np.flatnonzero(wb["alive"])
    cs = _cell(P, sb["x"][live_s], sb["y"][live_s])
    cw = _cell(P, wb["x"][live_w], wb["y"][live_w])
    exp_e_s = sb["e"].copy()
    exp_alive_s = sb["alive"].copy()
    exp_e_w = wb["e"].copy()
    exp_grass = before.grass.copy()
    n_grass = n_prey = 0
    by_cell_s = {}
    for i, c in zip(live_s, cs):
        by_cell_s.setdefault(int(c), []).append(int(i))
    by_cell_w = {}
    for j, c in zip(live_w, cw):
        by_cell_w.setdefault(int(c), []).append(int(j))
    for c, sheep in by_cell_s.items():
        if before.grass[c] == 0:
            w = min(sheep, key=lambda i: _key(orc, P, t, i, 0x14))
            exp_e_s[w] += P.gain_s
            exp_grass[c] = P.R
            n_grass += 1
    for c, sheep in by_cell_s.items():
        if c not in by_cell_w:
            continue
        if P.multi_prey:
            # the r-th sheep (by prey key) of the cell is eaten by its r-th wolf (by eat key)
            prey_order = sorted(sheep, key=lambda i: _key(orc, P, t, i, 0x15))
            wolf_order = sorted(by_cell_w[c], key=lambda j: _key(orc, P, t, j, 0x24))
            pairs = list(zip(prey_order, wolf_order))
        else:
            pairs = [(min(sheep, key=lambda i: _key(orc, P, t, i, 0x15)),
                      min(by_cell_w[c], key=lambda j: _key(orc, P, t, j, 0x24)))]
        for prey, wolf in pairs:
            exp_alive_s[prey] = 0
            exp_e_w[wolf] += P.gain_w
            n_prey += 1
    assert (ng, ns) == (n_grass, n_prey)
    assert np.array_equal(sa["e"], exp_e_s) and np.array_equal(sa["alive"], exp_alive_s)
    assert np.array_equal(wa["e"], exp_e_w) and np.array_equal(wa["alive"], wb["alive"])
    assert np.array_equal(after.grass, exp_grass)
    for f in ("x", "y"):
        assert np.array_equal(sa[f], sb[f]) and np.array_equal(wa[f], wb[f])
    assert ng <= G and ns <= min(live_s.size, live_w.size)
    if not P.multi_prey:
        assert ns <= G


def _check_breed(orc, P, before, after, t, bs, bw):
    for sp, purpose, T, cap, births in (("sheep", 0x16, P.T_s, P.cap_s, bs),
                                        ("wolves", 0x26, P.T_w, P.cap_w, bw)):
        b, a = getattr(before, sp), getattr(after, sp)
        elig = [i for i in range(cap)
                if b["alive"][i] and b["e"][i] > 0 and orc.rng(P.seed, t, i, purpose) < T]
        free = np.flatnonzero(b["alive"] == 0)
        r = min(len(elig), free.size)
        assert births == r
        # children: the r lowest free slots, on the parent's cell, energy conserved
        for j in range(r):
            par, ch = elig[j], int(free[j])
            assert a["alive"][ch] == 1
            assert (a["x"][ch], a["y"][ch]) == (b["x"][par], b["y"][par])
            assert a["e"][ch] + a["e"][par] == b["e"][par]
            assert a["e"][ch] == b["e"][par] // 2
        assert np.all(a["alive"][free[r:]] == 0)
        touched = set(elig[:r]) | set(int(c) for c in free[:r])
        rest = np.array([i for i in range(cap) if i not in touched], dtype=np.int64)
        for f in FIELDS:
            assert np.array_equal(a[f][rest], b[f][rest])
        live_b, live_a = b["alive"] != 0, a["alive"] != 0
        assert int(a["e"][live_a].sum()) == int(b["e"][live_b].sum())


def _check_die(P, before, after, ss, sw):
    for sp, n in (("sheep", ss), ("wolves", sw)):
        b, a = getattr(before, sp), getattr(after, sp)
        dying = (b["alive"] != 0) & (b["e"] < 0)
        assert n == int(dying.sum())
        assert np.all(a["alive"][dying] == 0)
        assert np.array_equal(a["alive"][~dying], b["alive"][~dying])
        for f in ("x", "y", "e"):
            assert np.array_equal(a[f], b[f])


def _check_regrow(P, before, after):
    assert np.array_equal(after.grass, np.maximum(before.grass - 1, 0))


def _phase_checked_step(orc, P, S):
    t = S.step
    live_s0 = int(np.count_nonzero(S.sheep["alive"]))
    live_w0 = int(np.count_nonzero(S.wolves["alive"]))
    s0 = S.copy()
    orc.pred_move(P, S)
    _check_move(orc, P, s0, S, t)
    s1 = S.copy()
    ng, ns = orc.pred_eat(P, S)
    _check_eat(orc, P, s1, S, t, ng, ns)
    s2 = S.copy()
    bs, bw = orc.pred_breed(P, S)
    _check_breed(orc, P, s2, S, t, bs, bw)
    s3 = S.copy()
    ss, sw = orc.pred_die(P, S)
    _check_die(P, s3, S, ss, sw)
    s4 = S.copy()
    orc.pred_regrow(P, S)
    _check_regrow(P, s4, S)
    S.step = t + 1
    # population bookkeeping of the whole step
    assert np.count_nonzero(S.sheep["alive"]) == live_s0 - ns - ss + bs
    assert np.count_nonzero(S.wolves["alive"]) == live_w0 - sw + bw
    assert 0 <= S.grass.min() and S.grass.max() <= P.R - 1
    if t >= 1:
        assert int(np.count_nonzero(S.grass == P.R - 1)) == ng
    for sp in SPECIES:
        d = getattr(S, sp)
        live = d["alive"] != 0
        assert np.all((d["x"][live] >= 0) & (d["x"][live] < P.W))
        assert np.all((d["y"][live] >= 0) & (d["y"][live] < P.H))
        assert set(np.unique(d["alive"])) <= {0, 1}
    return dict(live_s=live_s0, live_w=live_w0, grass_eaten=ng, sheep_eaten=ns,
                births_s=bs, births_w=bw, starved_s=ss, starved_w=sw)


@pytest.mark.parametrize("multi_prey", [0, 1])
@pytest.mark.parametrize("W,H,cap_s,cap_w,n_s0,n_w0,seeds,steps", [
    (1, 1, 6, 4, 3, 2, range(0, 40), 6),      # every agent on one cell: all conflicts
    (2, 1, 6, 4, 4, 2, range(40, 70), 6),
    (3, 3, 8, 6, 5, 3, range(70, 90), 8),
    (8, 8, 64, 16, 20, 6, range(90, 94), 12),
])
def test_phase_invariants_tiny(orc, W, H, cap_s, cap_w, n_s0, n_w0, seeds, steps, multi_prey):
    for seed in seeds:
        P = orc.pred_params(W=W, H=H, R=3, T_s=2**31, T_w=2**31, seed=seed,
                            cap_s=cap_s, cap_w=cap_w, n_s0=n_s0, n_w0=n_w0,
                            multi_prey=multi_prey)
        S = orc.predation_init(P)
        ref = S.copy()
        for _ in range(steps):
            st = _phase_checked_step(orc, P, S)
            assert orc.predation_step(P, ref) == st
        for sp in SPECIES:
            for f in FIELDS:
                assert np.array_equal(getattr(S, sp)[f], getattr(ref, sp)[f])
        assert np.array_equal(S.grass, ref.grass)


def test_phase_invariants_small_workload(orc):
    """The 64x64 workload (400 sheep, 100 wolves) for its first 12 steps."""
    P = orc.pred_params(seed=3)
    S = orc.predation_init(P)
    for _ in range(12):
        _phase_checked_step(orc, P, S)


def test_init_distribution(orc):
    P = orc.pred_params(W=64, H=64, seed=1)
    S = orc.predation_init(P)
    grown = float(np.mean(S.grass == 0))
    assert abs(grown - 0.5) < 0.03
    cd = S.grass[S.grass > 0]
    assert cd.min() >= 1 and cd.max() <= P.R
    assert np.all(S.sheep["alive"][:400] == 1) and np.all(S.sheep["alive"][400:] == 0)
    assert np.all(S.wolves["alive"][:100] == 1) and np.all(S.wolves["alive"][100:] == 0)
    assert S.sheep["e"][:400].min() >= 0 and S.sheep["e"][:400].max() < 8
    assert S.wolves["e"][:100].min() >= 0 and S.wolves["e"][:100].max() < 40
    for f in FIELDS:
        assert not S.sheep[f][400:].any() and not S.wolves[f][100:].any()


def test_starvation_special_case(orc):
    """A lone sheep with zero energy on an ungrown 1x1 cell pays the move cost,
    cannot breed (energy not positive) and dies; its fields stay stale."""
    P = orc.pred_params(W=1, H=1, R=9, cap_s=2, cap_w=1, n_s0=0, n_w0=0, T_s=2**32 - 1)
    S = orc.predation_init(P)
    S.grass[:] = 5
    S.sheep["alive"][0] = 1
    S.sheep["e"][0] = 0
    st = orc.predation_step(P, S)
    assert st["starved_s"] == 1 and st["births_s"] == 0 and st["grass_eaten"] == 0
    assert list(S.sheep["alive"]) == [0, 0] and S.sheep["e"][0] == -1
    assert list(S.grass) == [4]


def test_regrowth_timing(orc):
    """A cell eaten at step t is edible again exactly at step t + R."""
    R = 4
    P = orc.pred_params(W=1, H=1, R=R, cap_s=1, cap_w=1, n_s0=0, n_w0=0, T_s=0)
    S = orc.predation_init(P)
    S.grass[:] = 0
    S.sheep["alive"][0] = 1
    S.sheep["e"][0] = 1000
    eaten_at = [t for t in range(13) if orc.predation_step(P, S)["grass_eaten"]]
    assert eaten_at == [0, R, 2 * R, 3 * R]


def test_capacity_never_exceeded_and_overflow_dropped(orc):
    P = orc.pred_params(W=4, H=4, cap_s=10, cap_w=4, n_s0=10, n_w0=4, T_s=2**32 - 1,
                        T_w=2**32 - 1, seed=2)
    S = orc.predation_init(P)
    for _ in range(20):
        st = orc.predation_step(P, S)
        assert np.count_nonzero(S.sheep["alive"]) <= P.cap_s
        assert st["births_s"] <= P.cap_s - (st["live_s"] - st["sheep_eaten"])


def test_determinism_and_resume(orc):
    """Same seed -> identical bytes; 30 steps straight equals 15 + copy + 15,
    because the draws are keyed on (seed, step) and no RNG state is carried."""
    P = orc.pred_params(seed=17)
    a = orc.predation_init(P)
    b = orc.predation_init(P)
    orc.predation_run(P, a, 30)
    orc.predation_run(P, b, 15)
    c = b.copy()
    orc.predation_run(P, c, 15)
    assert c.step == a.step == 30
    assert np.array_equal(a.grass, c.grass)
    for sp in SPECIES:
        for f in FIELDS:
            assert np.array_equal(getattr(a, sp)[f], getattr(c, sp)[f])


def test_small_workload_population_oscillates(orc):
    """Qualitative only (Fig. 3 shows no numbers): both species persist for
    200 steps on most seeds and the sheep count is not monotone."""
    persisted = 0
    for seed in range(5):
        P = orc.pred_params(seed=seed)
        S = orc.predation_init(P)
        st = orc.predation_run(P, S, 200)
        live_s = [s["live_s"] for s in st]
        persisted += live_s[-1] > 0
        assert max(live_s) > min(live_s)
    assert persisted >= 3


def _eat_both_ways(orc, P, S):
    a, b = S.copy(), S.copy()
    P1 = orc.pred_params(**{f: getattr(P, f) for f, _ in P._fields_ if f != "multi_prey"},
                         multi_prey=1)
    ra = orc.pred_eat(P, a)
    rb = orc.pred_eat(P1, b)
    return a, b, ra, rb


def test_multi_prey_reduces_to_one_prey_rule(orc):
    """With at most one wolf or at most one sheep on every cell, pairing by rank
    eats exactly what the one-prey rule eats (the rule the rest of the model,
    and the GPU path, is pinned on)."""
    g = np.random.default_rng(5)
    checked = 0
    for trial in range(300):
        P = orc.pred_params(W=6, H=5, seed=int(g.integers(0, 2**32)), cap_s=40, cap_w=12,
                            n_s0=0, n_w0=0)
        S = orc.predation_init(P)
        S.step = int(g.integers(0, 1000))
        ns, nw = int(g.integers(0, 40)), int(g.integers(0, 12))
        cells_w = g.choice(30, size=nw, replace=False) if trial % 2 else g.integers(0, 30, nw)
        cells_s = g.integers(0, 30, ns) if trial % 2 else g.choice(30, size=min(ns, 30), replace=False)
        for sp, cells in (("sheep", cells_s), ("wolves", cells_w)):
            d = getattr(S, sp)
            for i, c in enumerate(cells):
                d["x"][i], d["y"][i], d["alive"][i], d["e"][i] = c % 6, c // 6, 1, 5
        a, b, ra, rb = _eat_both_ways(orc, P, S)
        assert ra == rb
        for sp in SPECIES:
            for f in FIELDS:
                assert np.array_equal(getattr(a, sp)[f], getattr(b, sp)[f])
        checked += 1
    assert checked == 300


def test_multi_prey_worked_cell(orc):
    """One cell, keys ordered by hand in tests/golden/predation_multi_prey_1x1.txt:
    (a) four sheep and three wolves, (b) two sheep and three wolves."""
    meta, exp = {}, {}
    for line in open(golden_path("predation_multi_prey_1x1.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        key, val = line.split(":", 1)
        if key == "params":
            meta = {k: int(v) for k, v in (t.split("=") for t in val.split())}
        else:
            exp[key] = [int(v) for v in val.split()]
    P = orc.pred_params(**meta)
    for case, n_s, e_w in (("a", 4, [7, 7, 7]), ("b", 2, [7, 8, 9])):
        S = orc.predation_init(P)
        S.step = exp["step"][0]
        for sp, n in (("sheep", n_s), ("wolves", 3)):
            d = getattr(S, sp)
            d["alive"][:] = 0
            d["alive"][:n] = 1
            d["x"][:] = 0
            d["y"][:] = 0
            d["e"][:n] = 7
        S.wolves["e"][:3] = e_w
        ng, ns = orc.pred_eat(P, S)
        assert ns == min(n_s, 3), case
        assert list(S.sheep["alive"]) == exp[f"{case}.sheep_alive_after"], case
        assert list(S.wolves["e"]) == exp[f"{case}.wolf_e_after"], case


def test_move_every_direction_worked_by_hand(orc):
    """Every one of the eight move directions (Sec. 5.1, Fig. 2), each with its
    exact displacement, including wraps in x, in y and in both, on a 5x5
    torus worked by hand (tests/golden/predation_moves_8dirs.txt).  Swapping
    any two entries of the direction table, or dropping the wrap, fails here."""
    meta, exp = _load_hand("predation_moves_8dirs.txt")
    P = orc.pred_params(**meta)
    S = orc._empty_state(P)
    for sp in SPECIES:
        for f in FIELDS:
            getattr(S, sp)[f][:] = exp[f"before.{sp}.{f}"]
    S.step = 0
    # the draws of the fixture are the oracle's draws for this seed and step
    for sp, purpose in (("sheep", 0x13), ("wolves", 0x23)):
        dirs = [orc.rng(P.seed, 0, i, purpose) >> 29 for i in range(8)]
        assert dirs == exp[f"draws.{sp}"], sp
    assert sorted(exp["draws.sheep"]) == list(range(8))
    orc.pred_move(P, S)
    for sp in SPECIES:
        for f in FIELDS:
            assert list(getattr(S, sp)[f]) == exp[f"after.{sp}.{f}"], f"{sp}.{f}"
    # each live agent's displacement is the table entry of its draw
    for sp in SPECIES:
        live = np.flatnonzero(np.array(exp[f"before.{sp}.alive"]))
        for i in live:
            d = exp[f"draws.{sp}"][i]
            dx = (exp[f"after.{sp}.x"][i] - exp[f"before.{sp}.x"][i]) % P.W
            dy = (exp[f"after.{sp}.y"][i] - exp[f"before.{sp}.y"][i]) % P.H
            assert dx == exp["dirs.dx"][d] % P.W and dy == exp["dirs.dy"][d] % P.H, (sp, i, d)
