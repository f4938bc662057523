"""Pins for the oracle's traffic cellular automaton (Sec. 5.2, Fig. 4).

The paper describes the model's ingredients but prints no trajectories, so
the oracle is pinned by (i) four steps worked by hand on a 3 x 4 road,
(ii) a per-step check over many seeds that re-derives every car's outcome
from the start-of-step state and the draws (exit under a green light,
blocked by an occupied target, the conflict winner by the cell's priority
mask, spawning into free entry cells and the lowest free slots), and
(iii) special cases (no spawning, a permanent red light, a permanent green).
"""
import numpy as np
import pytest

from conftest import golden_path

LIGHT, LANE, SPAWN = 0x30, 0x31, 0x32


def _load(name):
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


def test_hand_worked_steps(orc):
    meta, exp = _load("traffic_hand_L4.txt")
    P = orc.traffic_params(**meta)
    S = orc.TrafficState(*(np.array(exp[f"start.{f}"], dtype=np.int32)
                           for f in ("lane", "pos", "alive")), exp["start.step"][0])
    for t in range(4, 8):
        assert orc.traffic_step(P, S) == exp[f"stats.{t}"], t
        for f in ("lane", "pos", "alive"):
            assert list(getattr(S, f)) == exp[f"after.{t}.{f}"], (t, f)


def _expected_step(orc, P, S):
    """Every car's outcome re-derived from the start-of-step state."""
    L, t, n = P.length, S.step, 3 * P.length
    occ = {}
    for i in np.flatnonzero(S.alive):
        occ[(int(S.lane[i]), int(S.pos[i]))] = int(i)
    green = [orc.rng(P.seed, t, l, LIGHT) < P.T_green for l in range(3)]
    leave, claims, stats = set(), {}, dict(cars=len(occ), exited=0, moved=0, blocked=0, lost=0,
                                           waiting_red=0, spawned=0, lane_changes=0)
    for (l, x), i in occ.items():
        if x == L - 1:
            if green[l]:
                leave.add(i)
            else:
                stats["waiting_red"] += 1
            continue
        nl = l + orc.uniform(orc.rng(P.seed, t, i, LANE), 3) - 1
        if not 0 <= nl <= 2:
            nl = l
        if (nl, x + 1) in occ:
            stats["blocked"] += 1
            continue
        prio = 0 if nl == l else (1 if l < nl else 2)
        claims.setdefault((nl, x + 1), []).append((prio, i))
    lane, pos, alive = S.lane.copy(), S.pos.copy(), S.alive.copy()
    for cell, cl in claims.items():
        prios = [p for p, _ in cl]
        assert len(set(prios)) == len(prios)        # one claimant per incoming direction
        _, w = min(cl)
        stats["moved"] += 1
        stats["lost"] += len(cl) - 1
        stats["lane_changes"] += int(lane[w] != cell[0])
        lane[w], pos[w] = cell
    for i in leave:
        alive[i] = 0
    stats["exited"] = len(leave)
    occupied_entry = {int(lane[i]) for i in np.flatnonzero(alive) if pos[i] == 0}
    spawn = [l for l in range(3)
             if l not in occupied_entry and orc.rng(P.seed, t, l, SPAWN) < P.T_spawn]
    free = [int(i) for i in range(n) if alive[i] == 0]
    for l, i in zip(spawn, free):
        lane[i], pos[i], alive[i] = l, 0, 1
    stats["spawned"] = min(len(spawn), len(free))
    return lane, pos, alive, stats


@pytest.mark.parametrize("length,T_green,T_spawn", [
    (2, 2 ** 31, 2 ** 31), (3, 2 ** 30, 3 * 2 ** 30), (7, 2 ** 31, 2 ** 31),
    (12, 3 * 2 ** 30, 2 ** 30), (40, 2 ** 31, 3 * 2 ** 30),
])
def test_every_step_rederived(orc, length, T_green, T_spawn):
    for seed in range(25):
        P = orc.traffic_params(length=length, T_green=T_green, T_spawn=T_spawn, seed=seed)
        S = orc.traffic_init(P)
        for _ in range(30):
            lane, pos, alive, st = _expected_step(orc, P, S)
            got = orc.traffic_step(P, S)
            assert got == st
            assert np.array_equal(S.alive, alive)
            live = alive != 0
            assert np.array_equal(S.lane[live], lane[live]) and np.array_equal(S.pos[live], pos[live])
            cells = set(zip(S.lane[live].tolist(), S.pos[live].tolist()))
            assert len(cells) == int(live.sum())       # one car per cell
            assert got["cars"] - got["exited"] + got["spawned"] == int(live.sum())


def test_no_spawning_keeps_the_road_empty(orc):
    P = orc.traffic_params(length=10, T_spawn=0, seed=4)
    S = orc.traffic_init(P)
    for st in orc.traffic_run(P, S, 50):
        assert st["cars"] == 0 and st["spawned"] == 0
    assert not S.alive.any()


def test_permanent_red_fills_the_road(orc):
    """No car can leave: the road fills cell by cell until every slot is a car
    that cannot move."""
    P = orc.traffic_params(length=6, T_green=0, T_spawn=2 ** 32 - 1, seed=2)
    S = orc.traffic_init(P)
    stats = orc.traffic_run(P, S, 200)
    assert all(st["exited"] == 0 for st in stats)
    assert S.alive.all()
    assert stats[-1]["moved"] == 0 and stats[-1]["spawned"] == 0
    assert stats[-1]["waiting_red"] == 3


def test_permanent_green_never_waits(orc):
    P = orc.traffic_params(length=5, T_green=2 ** 32 - 1, T_spawn=2 ** 32 - 1, seed=6)
    S = orc.traffic_init(P)
    stats = orc.traffic_run(P, S, 100)
    assert all(st["waiting_red"] == 0 for st in stats)
    assert sum(st["exited"] for st in stats) > 0
