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
        grass, sheep, wolves, updates = runner.result(q.rid)
        assert np.array_equal(grass, St.grass), q.rid
        for name, got, exp in (("sheep", sheep, St.sheep), ("wolves", wolves, St.wolves)):
            for f in ("x", "y", "e", "alive"):
                assert np.array_equal(got[f], exp[f]), (q.rid, name, f)
        assert updates == sum(s["live_s"] + s["live_w"] for s in st), q.rid


def test_stratified_sample_of_the_served_trace(abm, orc):
    """Requests of the served workload's own trace (Poisson 200/s over 60 s,
    side log-uniform in [32, 1024], steps log-uniform in [100, 5000]): from
    each of 16 side strata the request with the fewest steps (which bounds the
    oracle's time), and from each of 4 step-count strata the request with the
    smallest side (long runs), and the largest grid's shortest request;
    arrivals compressed 50x so they overlap on the device.
    Teams of 4 for models of at least 2^18 cells plus slots, as served.
    Every result equals the oracle's run of that request alone."""
    from paper_2508_16508_amd import workloads as W
    trace = W.served_trace(0)
    order = sorted(range(len(trace)), key=lambda i: trace[i].side)
    strata = np.array_split(np.asarray(order), 16)
    pick = {int(min(s, key=lambda i: trace[i].steps)) for s in strata}
    by_steps = sorted(range(len(trace)), key=lambda i: trace[i].steps)
    pick |= {int(min(s, key=lambda i: (trace[i].side, -trace[i].steps)))
             for s in np.array_split(np.asarray(by_steps), 4)}
    # and the request of side >= 1000 with the fewest steps (the largest grids)
    pick.add(min((i for i in range(len(trace)) if trace[i].side >= 1000),
                 key=lambda i: trace[i].steps))
    pick = sorted(pick)
    reqs = [S.Request(i, trace[i].arrival_s / 50.0, trace[i].side, trace[i].steps,
                      trace[i].seed) for i in pick]
    assert max(q.side for q in reqs) >= 1000 and min(q.side for q in reqs) < 40
    big = [q for q in reqs if q.cells + q.cap_s + q.cap_w >= 1 << 18]
    assert len(big) >= 3                       # the team path is exercised
    assert max(q.steps for q in reqs) > 3000
    cells = sum(q.cells for q in reqs)
    sheep, wolves = sum(q.cap_s for q in reqs), sum(q.cap_w for q in reqs)
    runner = S.GpuRunner(cells, sheep, wolves, keep_results=True, team_size=4,
                         team_min_size=1 << 18, max_model_cap=max(q.cap_s for q in reqs))
    sch = S.Scheduler(runner, cells, sheep, wolves)
    rep = sch.serve(reqs)
    assert rep.summary()["requests"] == len(reqs) and rep.max_active > 1
    assert runner.workspace_error == 0
    for q in reqs:
        P = orc.pred_params(W=q.side, H=q.side, seed=q.seed & 0xFFFFFFFF, cap_s=q.cap_s,
                            cap_w=q.cap_w, n_s0=q.n_s0, n_w0=q.n_w0)
        St = orc.predation_init(P)
        st = orc.predation_run(P, St, q.steps)
        grass, sheep_g, wolves_g, updates = runner.result(q.rid)
        assert np.array_equal(grass, St.grass), q.rid
        for name, got, exp in (("sheep", sheep_g, St.sheep), ("wolves", wolves_g, St.wolves)):
            for f in ("x", "y", "e", "alive"):
                assert np.array_equal(got[f], exp[f]), (q.rid, name, f)
        assert updates == sum(s["live_s"] + s["live_w"] for s in st), q.rid
