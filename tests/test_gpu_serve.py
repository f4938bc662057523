"""The served form on the GPU: requests that arrive while others run are
admitted into the running batch, and each result is bit-identical to the
same model run alone (the oracle), however it was interleaved."""
import numpy as np
import pytest
import torch

from paper_2508_16508_amd import serve as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("team_size", [1, 4])
def test_each_result_same_alone_and_in_the_mix(abm, orc, team_size):
    """team_size 4: models of at least 1200 cells plus slots run on teams."""
    g = np.random.default_rng(11)
    reqs = []
    t = 0.0
    for i in range(36):
        t += float(g.exponential(0.002))
        side = int(g.integers(4, 41))
        steps = int(g.integers(5, 80))
        reqs.append(S.Request(i, t, side, steps, int(g.integers(0, 2 ** 32))))
    cells = 6 * 40 * 40          # room for only a handful of models at once: requests queue
    runner = S.GpuRunner(cells, cells, cells // 2, keep_results=True, team_size=team_size,
                         team_min_size=1200)
    sch = S.Scheduler(runner, cells, cells, cells // 2, slot_step_budget=4000)
    rep = sch.serve(reqs)
    summ = rep.summary()
    assert summ["requests"] == 36 and summ["chunks"] > 5
    assert rep.max_active > 1
    for q in reqs:
        P = orc.pred_params(W=q.side, H=q.side, seed=q.seed, cap_s=q.cap_s, cap_w=q.cap_w,
                            n_s0=q.n_s0, n_w0=q.n_w0)
        St = orc.predation_init(P)
        st = orc.predation_run(P, St, q.steps)
        grass, sheep, wolves, updates = runner.results[q.rid]
        assert np.array_equal(grass, St.grass), q.rid
        for name, got, exp in (("sheep", sheep, St.sheep), ("wolves", wolves, St.wolves)):
            for f in ("x", "y", "e", "alive"):
                assert np.array_equal(got[f], exp[f]), (q.rid, name, f)
        assert updates == sum(s["live_s"] + s["live_w"] for s in st), q.rid
