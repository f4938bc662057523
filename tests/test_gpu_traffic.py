"""GPU parity of the traffic cellular automaton (Sec. 5.2) against the CPU
oracle: every road of a batch must match the oracle run alone with its own
seed (seed + road), slot by slot (lane, pos, alive, stale fields included)
and in every per-step statistic."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _check_roads(abm, orc, roads, stats, steps, roads_to_check=None):
    P = roads.params
    n = 3 * P.length
    lane, pos, alive = (t.cpu().numpy() for t in (roads.lane, roads.pos, roads.alive))
    st = stats.cpu().numpy()
    for r in (roads_to_check if roads_to_check is not None else range(roads.n_roads)):
        OP = orc.traffic_params(P.length, P.T_green, P.T_spawn, (P.seed + r) & 0xFFFFFFFF)
        S = orc.traffic_init(OP)
        exp = orc.traffic_run(OP, S, steps)
        e = np.array([[d[k] for k in orc.TRAFFIC_STATS] for d in exp])
        assert np.array_equal(st[:, r], e), f"stats of road {r}"
        assert np.array_equal(alive[r], S.alive), f"alive of road {r}"
        assert np.array_equal(lane[r], S.lane) and np.array_equal(pos[r], S.pos), f"road {r}"
    assert abm.TRAFFIC_STAT_NAMES == orc.TRAFFIC_STATS


def _run(abm, length, n_roads, chunks, **kw):
    roads = abm.TrafficRoads(abm.traffic_params(length, **kw), n_roads)
    roads.init()
    parts = []
    for c in chunks:
        s = torch.zeros((c, n_roads, 8), dtype=torch.int64, device="cuda")
        roads.run(c, s)
        parts.append(s)
    torch.cuda.synchronize()
    return roads, torch.cat(parts)


@pytest.mark.parametrize("length,n_roads,kw", [
    (100, 48, dict(seed=0)),
    (7, 40, dict(T_green=2 ** 30, T_spawn=3 * 2 ** 30, seed=5)),
    (2, 30, dict(T_green=3 * 2 ** 30, T_spawn=2 ** 32 - 1, seed=9)),
    (61, 20, dict(T_green=0, T_spawn=2 ** 32 - 1, seed=3)),       # a jam that fills the road
    (1024, 3, dict(T_spawn=3 * 2 ** 30, seed=12)),                 # the longest road
    (33, 10, dict(T_spawn=0, seed=4)),                             # never a car
])
def test_roads_match_oracle(abm, orc, length, n_roads, kw):
    roads, stats = _run(abm, length, n_roads, (50, 1, 99), **kw)
    assert roads.step == 150
    _check_roads(abm, orc, roads, stats, 150)


def test_table3_scale_sample(abm, orc):
    """500 roads of 3 x 100 cells for 1000 steps (the largest run of the
    paper's traffic table): 12 roads spread over the batch compared in full."""
    roads, stats = _run(abm, 100, 500, (1000,), seed=100)
    _check_roads(abm, orc, roads, stats, 1000, roads_to_check=range(0, 500, 43))
    st = stats.cpu().numpy()
    assert (st[1:, :, 0] == st[:-1, :, 0] - st[:-1, :, 1] + st[:-1, :, 6]).all()


def test_seed_wraps_per_road(abm, orc):
    roads, stats = _run(abm, 9, 4, (20,), seed=2 ** 32 - 2)
    _check_roads(abm, orc, roads, stats, 20)


def test_invalid_arguments_are_rejected(abm):
    for length in (1, 1025):
        roads = abm.TrafficRoads(abm.traffic_params(2), 1)
        roads.params = abm.traffic_params(length)
        with pytest.raises(abm.AbmError):
            roads.init()
    roads = abm.TrafficRoads(abm.traffic_params(5), 2)
    roads.init()
    with pytest.raises(abm.AbmError):
        roads.run(-1)
