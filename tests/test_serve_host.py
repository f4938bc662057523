"""Host logic of the served form, on the CPU: pool allocation, admission by
footprint, per-chunk step budgets, retirement and open-loop latency, driven
by a fake device runner and a fake clock."""
import numpy as np
import pytest

from paper_2508_16508_amd.serve import RangeAllocator, Request, Scheduler


def test_range_allocator_first_fit_and_coalescing():
    a = RangeAllocator(100)
    x = a.alloc(30)
    y = a.alloc(30)
    z = a.alloc(30)
    assert (x, y, z) == (0, 30, 60)
    assert a.alloc(20) is None
    a.free(y, 30)
    assert a.alloc(31) is None
    assert a.alloc(25) == 30
    a.free(x, 30)
    a.free(30, 25)
    a.free(z, 30)
    assert a.free_total == 100 and a.alloc(100) == 0


class FakeRunner:
    """Advances each model to its chunk target; each chunk costs simulated time
    proportional to the largest slot-steps of any model in it."""

    def __init__(self, clock):
        self.clock = clock
        self.inited = []
        self.finished = []
        self.live_ranges = {}
        self.submitted = self.collected = 0

    def init(self, models):
        for r in models:
            for name, off, n in (("c", r.cell_off, r.req.cells), ("s", r.sheep_off, r.req.cap_s),
                                 ("w", r.wolf_off, r.req.cap_w)):
                for (o2, n2, _) in [v for k, v in self.live_ranges.items() if k[0] == name]:
                    assert off + n <= o2 or o2 + n2 <= off, "overlapping allocation"
                self.live_ranges[(name, r.req.rid)] = (off, n, r.req.rid)
            self.inited.append(r.req.rid)

    def submit(self, models, targets, admitted):
        self.init(admitted)
        work = max((t - r.step) * (r.req.cap_s + r.req.cap_w) for r, t in zip(models, targets))
        self.clock.t += 1e-3 + work * 1e-9
        self.submitted += 1
        self.max_in_flight = max(getattr(self, "max_in_flight", 0),
                                 self.submitted - self.collected)
        return [(t, (t - r.step) * 10) for r, t in zip(models, targets)]

    def collect(self, ticket):
        self.collected += 1
        assert self.submitted - self.collected <= 1   # at most two chunks in flight
        return ticket

    def finish(self, r):
        self.finished.append(r.req.rid)
        for name in ("c", "s", "w"):
            del self.live_ranges[(name, r.req.rid)]


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _trace(n, seed, rate=200.0):
    g = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(n):
        t += float(g.exponential(1 / rate))
        side = int(round(np.exp(g.uniform(np.log(32), np.log(1024)))))
        steps = int(round(np.exp(g.uniform(np.log(100), np.log(5000)))))
        out.append(Request(i, t, side, steps, int(g.integers(0, 2 ** 32))))
    return out


def test_every_request_completes_once_with_its_steps():
    clock = FakeClock()
    run = FakeRunner(clock)
    reqs = _trace(300, 1)
    sch = Scheduler(run, 50_000_000, 20_000_000, 5_000_000, clock=clock, sleep=clock.sleep)
    rep = sch.serve(reqs)
    assert sorted(run.finished) == list(range(300)) == sorted(run.inited)
    assert sorted(c[0] for c in rep.completed) == list(range(300))
    for rid, lat, que, upd in rep.completed:
        assert lat >= 0 and 0 <= que <= lat
        assert upd == reqs[rid].steps * 10
    assert not run.live_ranges
    assert sch.cells.free_total == 50_000_000
    assert run.max_in_flight == 2     # the next chunk is submitted before the last is collected


def test_admission_waits_for_footprint():
    """With pools that hold one large model at a time, requests queue and
    their latency includes the wait."""
    clock = FakeClock()
    run = FakeRunner(clock)
    reqs = [Request(i, 0.001 * i, 1000, 200, i) for i in range(4)]
    sch = Scheduler(run, 1_100_000, 500_000, 200_000, clock=clock, sleep=clock.sleep)
    rep = sch.serve(reqs)
    assert rep.max_active == 1
    order = [c[0] for c in rep.completed]
    assert order == [0, 1, 2, 3]            # FIFO admission
    lats = [c[1] for c in rep.completed]
    assert lats == sorted(lats) and rep.completed[-1][2] > 0


def test_chunk_budget_small_models_finish_in_one_chunk():
    clock = FakeClock()
    run = FakeRunner(clock)
    sch = Scheduler(run, 10 ** 8, 10 ** 8, 10 ** 8, slot_step_budget=1 << 22, clock=clock,
                    sleep=clock.sleep)
    small = Request(0, 0.0, 32, 5000, 1)       # 512 slots: budget covers all 5000 steps
    big = Request(1, 0.0, 1024, 100, 2)        # 524k slots: 8 steps per chunk
    rep = sch.serve([small, big])
    assert rep.chunks == 13      # ceil(100 / 8); the small model finishes in chunk 1
    assert [c[0] for c in rep.completed] == [0, 1]


def test_request_that_can_never_fit_is_rejected():
    clock = FakeClock()
    sch = Scheduler(FakeRunner(clock), 100, 100, 100, clock=clock, sleep=clock.sleep)
    with pytest.raises(ValueError):
        sch.serve([Request(0, 0.0, 32, 10, 0)])


def test_team_models_get_the_budget_of_every_member():
    clock = FakeClock()

    class TeamRunner(FakeRunner):
        def workgroups_for(self, r):
            return 4 if r.req.side >= 500 else 1

    run = TeamRunner(clock)
    sch = Scheduler(run, 10 ** 8, 10 ** 8, 10 ** 8, slot_step_budget=1 << 22, clock=clock,
                    sleep=clock.sleep)
    big, small = Request(0, 0.0, 600, 5000, 1), Request(1, 0.0, 300, 5000, 2)
    from paper_2508_16508_amd.serve import Running
    rb, rs = Running(big, 0, 0, 0, 0.0), Running(small, 0, 0, 0, 0.0)
    assert sch.chunk_target(rb) == (4 << 22) // (big.cap_s + big.cap_w)
    assert sch.chunk_target(rs) == (1 << 22) // (small.cap_s + small.cap_w)


def test_one_chunk_in_flight_waits_for_each_chunk():
    clock = FakeClock()
    run = FakeRunner(clock)
    reqs = _trace(60, 2)
    sch = Scheduler(run, 50_000_000, 20_000_000, 5_000_000, clock=clock, sleep=clock.sleep,
                    depth=1)
    rep = sch.serve(reqs)
    assert sorted(c[0] for c in rep.completed) == list(range(60))
    assert run.max_in_flight == 1
