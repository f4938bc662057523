"""Served predation: continuous batching of simulation requests on one GPU.

Requests (a predation model: grid side, step count, seed) arrive over time.
Each is admitted when its footprint fits the device-resident pools, advanced
inside the running batched launch alongside every other admitted model, and
retired when it reaches its step count; new arrivals join at the next chunk
boundary.  Latency is measured open-loop: completion minus the request's
scheduled arrival time.

The model state of every request lives in three pools in HBM (cells: regrowth
step + three claim words; sheep slots; wolf slots).  A request takes one range
of each pool (first fit) for its lifetime, so admission is by HBM footprint.

The scheduling logic (Scheduler) is pure host code with an injectable clock
and device runner, so it is tested without a GPU; GpuRunner drives libabm.
"""
from __future__ import annotations

import bisect
import ctypes as C
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

# Model definition shared by every request (the small workload's parameters).
R_REGROW, GAIN_S, GAIN_W = 30, 4, 20
T_SHEEP, T_WOLF = 171798691, 214748364


class RangeAllocator:
    """First-fit allocator of [offset, offset + n) ranges in [0, capacity)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self._free = [(0, self.capacity)]    # sorted, coalesced (start, length)

    @property
    def free_total(self) -> int:
        return sum(n for _, n in self._free)

    def alloc(self, n: int):
        n = max(1, int(n))
        for i, (s, ln) in enumerate(self._free):
            if ln >= n:
                if ln == n:
                    self._free.pop(i)
                else:
                    self._free[i] = (s + n, ln - n)
                return s
        return None

    def free(self, start: int, n: int):
        n = max(1, int(n))
        i = bisect.bisect_left(self._free, (start, 0))
        self._free.insert(i, (start, n))
        # coalesce with neighbours
        merged = []
        for s, ln in self._free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((s, ln))
        self._free = merged


@dataclass
class Request:
    rid: int
    arrival_s: float
    side: int
    steps: int
    seed: int

    @property
    def cells(self) -> int:
        return self.side * self.side

    @property
    def n_s0(self) -> int:
        return self.cells // 10

    @property
    def n_w0(self) -> int:
        return self.cells // 40

    @property
    def cap_s(self) -> int:
        return max(1, 4 * self.n_s0)

    @property
    def cap_w(self) -> int:
        return max(1, 4 * self.n_w0)


@dataclass
class Running:
    req: Request
    cell_off: int
    sheep_off: int
    wolf_off: int
    admit_s: float
    step: int = 0
    updates: int = 0


@dataclass
class Report:
    completed: list = field(default_factory=list)   # (rid, latency_s, queue_s, updates)
    start_s: float = 0.0
    end_s: float = 0.0
    chunks: int = 0
    max_active: int = 0
    device_busy_s: float = None   # device time of the chunks, when the runner measures it

    def summary(self) -> dict:
        lat = np.array([c[1] for c in self.completed]) if self.completed else np.zeros(1)
        que = np.array([c[2] for c in self.completed]) if self.completed else np.zeros(1)
        upd = sum(c[3] for c in self.completed)
        span = max(1e-9, self.end_s - self.start_s)
        return {"requests": len(self.completed), "agent_updates": int(upd),
                "agent_updates_per_s": upd / span, "wall_s": span,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_queue_s": float(que.mean()), "chunks": self.chunks,
                "max_active": self.max_active,
                "device_idle_fraction": (None if self.device_busy_s is None
                                         else max(0.0, 1.0 - self.device_busy_s / span))}


class Scheduler:
    """Continuous batching over pooled device state, pipelined two chunks deep.

    runner: object with submit(models, targets, admitted) -> ticket (enqueues,
    without waiting, the initial state of `admitted` and one chunk advancing
    each model to its target step), collect(ticket) -> list of (step, updates
    made in that chunk) per model (waits for that chunk), finish(model) (the
    model's last chunk has been submitted; its state ranges are then reused
    by later chunks) and optionally workgroups_for(model); clock: a callable
    returning seconds since the start of the trace.

    A chunk advances every model to exactly its target, so the host knows
    which models a chunk completes as soon as it submits it: it frees their
    ranges, admits waiting requests into them and submits the next chunk while
    the previous one still runs on the device (the device orders the next
    chunk's initial states after it).  It then waits for the older chunk only,
    so the device always has the next chunk queued while the host plans."""

    def __init__(self, runner, cell_capacity, sheep_capacity, wolf_capacity, max_active=4096,
                 slot_step_budget=1 << 23, clock=None, sleep=None, log=None, log_every_s=5.0,
                 depth=2):
        self.runner = runner
        self.depth = depth          # chunks in flight (1: wait for each chunk before the next)
        self.cells = RangeAllocator(cell_capacity)
        self.sheep = RangeAllocator(sheep_capacity)
        self.wolves = RangeAllocator(wolf_capacity)
        self.max_active = max_active
        self.budget = slot_step_budget
        t0 = time.perf_counter()
        self.clock = clock or (lambda: time.perf_counter() - t0)
        self.sleep = sleep or time.sleep
        self.log = log
        self.log_every_s = log_every_s

    def fits(self, req: Request) -> bool:
        return (req.cells <= self.cells.capacity and req.cap_s <= self.sheep.capacity and
                req.cap_w <= self.wolves.capacity)

    def _admit(self, req: Request, now: float):
        c = self.cells.alloc(req.cells)
        if c is None:
            return None
        s = self.sheep.alloc(req.cap_s)
        if s is None:
            self.cells.free(c, req.cells)
            return None
        w = self.wolves.alloc(req.cap_w)
        if w is None:
            self.cells.free(c, req.cells)
            self.sheep.free(s, req.cap_s)
            return None
        return Running(req, c, s, w, now)

    def _release(self, r: Running):
        self.cells.free(r.cell_off, r.req.cells)
        self.sheep.free(r.sheep_off, r.req.cap_s)
        self.wolves.free(r.wolf_off, r.req.cap_w)

    def chunk_target(self, r: Running) -> int:
        """Steps this model may advance in the next chunk: a budget of slot-steps
        per workgroup, split by the model's slot count, so small models run many
        steps and large ones few, and a chunk's duration stays bounded.  A model
        advanced by a team of workgroups (runner.workgroups_for) gets the budget
        of every member."""
        wg = self.runner.workgroups_for(r) if hasattr(self.runner, "workgroups_for") else 1
        k = max(1, self.budget * wg // (r.req.cap_s + r.req.cap_w))
        return min(r.req.steps, r.step + k)

    def serve(self, requests) -> Report:
        pending = sorted(requests, key=lambda q: q.arrival_s)
        for q in pending:
            if not self.fits(q):
                raise ValueError(f"request {q.rid} can never fit the pools")
        waiting: list = []
        active: list = []          # models with steps still to submit
        inflight = deque()         # (ticket, models of the chunk, models it completes)
        rep = Report(start_s=self.clock())
        nxt = 0
        next_log = rep.start_s + self.log_every_s
        while nxt < len(pending) or waiting or active or inflight:
            now = self.clock()
            while nxt < len(pending) and pending[nxt].arrival_s <= now:
                waiting.append(pending[nxt])
                nxt += 1
            if not active and not waiting and not inflight:
                self.sleep(max(0.0, pending[nxt].arrival_s - now))
                continue
            admitted, still = [], []
            for q in waiting:   # FIFO; a request that does not fit waits
                r = self._admit(q, now) if len(active) + len(admitted) < self.max_active else None
                if r is None:
                    still.append(q)
                else:
                    admitted.append(r)
            waiting = still
            active.extend(admitted)
            if active and len(inflight) < self.depth:
                targets = [self.chunk_target(r) for r in active]
                ticket = self.runner.submit(active, targets, admitted)
                rep.chunks += 1
                rep.max_active = max(rep.max_active, len(active))
                done, keep = [], []
                for r, t in zip(active, targets):
                    r.step = t
                    (done if t >= r.req.steps else keep).append(r)
                for r in done:
                    self.runner.finish(r)
                    self._release(r)
                inflight.append((ticket, list(active), done))
                active = keep
                if len(inflight) < self.depth and (active or waiting):
                    continue       # plan the next chunk while this one runs
            elif not inflight:
                # nothing fits until something retires; cannot happen with nothing in flight
                raise RuntimeError("pools too small for the waiting requests")
            ticket, models, done = inflight.popleft()
            results = self.runner.collect(ticket)
            now = self.clock()
            for r, (step, updates) in zip(models, results):
                r.updates += updates
            for r in done:
                rep.completed.append((r.req.rid, now - r.req.arrival_s,
                                      r.admit_s - r.req.arrival_s, r.updates))
            if self.log and now >= next_log:
                next_log = now + self.log_every_s
                self.log(f"t={now:7.2f}s arrived={nxt} waiting={len(waiting)} "
                         f"active={len(active)} done={len(rep.completed)} chunks={rep.chunks}")
        rep.end_s = self.clock()
        rep.device_busy_s = getattr(self.runner, "busy_s", None)
        return rep


class GpuRunner:
    """Device side of the scheduler: pooled state and the batched launches."""

    def __init__(self, cell_capacity, sheep_capacity, wolf_capacity, max_active=4096,
                 block_threads=512, items=4, device="cuda", keep_results=False,
                 max_model_cap=None, team_size=4, team_min_size=1 << 18, lds=True):
        import torch

        import paper_2508_16508_amd as abm
        self.abm, self.torch = abm, torch
        z = lambda n: torch.zeros(max(1, n), dtype=torch.int32, device=device)
        self.ready = z(cell_capacity)
        self.claims = torch.full((3 * max(1, cell_capacity),), -1, dtype=torch.int64,
                                 device=device).view(torch.uint64)
        self.sheep = {f: z(sheep_capacity) for f in ("x", "y", "e", "alive")}
        self.wolves = {f: z(wolf_capacity) for f in ("x", "y", "e", "alive")}
        self.max_active = max_active
        self.desc_size = C.sizeof(abm.ModelDesc)
        self.desc = torch.zeros(max_active * self.desc_size, dtype=torch.uint8, device=device)
        self.init_desc = torch.zeros(max_active * self.desc_size, dtype=torch.uint8, device=device)
        self.order = torch.zeros(max_active, dtype=torch.int32, device=device)
        self.block_threads, self.items = block_threads, items
        # models of at least team_min_size cells plus slots run on teams of workgroups
        self.team_size, self.team_min_size = team_size, team_min_size
        # models of one workgroup whose claim table fits keep it in LDS
        self.lds = lds
        props = torch.cuda.get_device_properties(self.ready.device)
        self.workgroups = props.multi_processor_count * max(1, 2048 // block_threads)
        # breeder scratch per workgroup is sized by the largest single model
        self.max_cap = int(max_model_cap or max(sheep_capacity, wolf_capacity))
        nbytes = int(abm.lib().abm_batched_workspace_bytes(self.max_cap, self.workgroups))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off: off + nbytes]
        # zeroed once: the error word of the header is sticky
        abm._check(abm.lib().abm_workspace_init(abm._p(self.ws), nbytes, abm._stream()))
        self.keep_results = keep_results
        self.results = {}
        self.device = device
        self.workspace_error = 0
        # pinned host staging, one set per chunk in flight
        pin = lambda n, dt=torch.uint8: [torch.empty(n, dtype=dt, pin_memory=True) for _ in range(2)]
        self.h_desc = pin(max_active * self.desc_size)
        self.h_init = pin(max_active * self.desc_size)
        self.h_out = pin(max_active * self.desc_size)
        self.h_order = pin(max_active, torch.int32)
        self.h_err = pin(8)
        self._k = 0
        self.busy_s = 0.0      # device time of the chunks' batched launches

    def _team_model(self, r) -> bool:
        return self.team_size > 1 and r.req.cells + r.req.cap_s + r.req.cap_w >= self.team_min_size

    def workgroups_for(self, r) -> int:
        """Workgroups that will advance model r (a team, or one)."""
        return self.team_size if self._team_model(r) else 1

    def _descs(self, models, targets, zero=False):
        """Descriptors for a chunk: each model at its (planned) step, advancing
        to its target; updates start at 0, so the readback holds the chunk's
        own count.  zero: step 0, for the initial state."""
        abm = self.abm
        arr = (abm.ModelDesc * max(1, len(models)))()
        for i, r in enumerate(models):
            q, d = r.req, arr[i]
            d.W = d.H = q.side
            d.R, d.gain_s, d.gain_w = R_REGROW, GAIN_S, GAIN_W
            d.T_s, d.T_w, d.seed = T_SHEEP, T_WOLF, q.seed & 0xFFFFFFFF
            d.cap_s, d.cap_w, d.n_s0, d.n_w0 = q.cap_s, q.cap_w, q.n_s0, q.n_w0
            d.cell_off, d.sheep_off, d.wolf_off = r.cell_off, r.sheep_off, r.wolf_off
            d.step, d.steps_target = (0, 0) if zero else (r.step, targets[i])
            d.updates = 0
        return arr

    def _batch(self, desc_tensor, n):
        abm = self.abm
        sp = lambda d: abm.SpeciesPtrs(*(d[k].data_ptr() for k in ("x", "y", "e", "alive")))
        return abm.Batch(n, self.max_cap, desc_tensor.data_ptr(), self.ready.data_ptr(),
                         self.claims.data_ptr(), sp(self.sheep), sp(self.wolves))

    def _stage(self, host, arr, n):
        """Copies the first n descriptors of arr into the pinned host buffer."""
        raw = np.frombuffer(bytes(arr), dtype=np.uint8)[: n * self.desc_size]
        host.numpy()[: n * self.desc_size] = raw
        return host[: n * self.desc_size]

    def submit(self, models, targets, admitted):
        """Enqueues, without waiting: the initial state of the admitted models,
        one chunk advancing every model to its target step, and the readback
        of the descriptors and the error word.  Host buffers alternate between
        the two chunks in flight; the device buffers are reused in stream order
        (a chunk's uploads run after the previous chunk and its readback)."""
        abm, torch = self.abm, self.torch
        slot = self._k % 2
        self._k += 1
        stream = torch.cuda.current_stream()
        if admitted:
            na = len(admitted)
            h = self._stage(self.h_init[slot], self._descs(admitted, [0] * na, zero=True), na)
            self.init_desc[: h.numel()].copy_(h, non_blocking=True)
            b = self._batch(self.init_desc, na)
            abm._check(abm.lib().abm_predation_batched_init(C.byref(b), abm._stream()))
        n = len(models)
        h = self._stage(self.h_desc[slot], self._descs(models, targets), n)
        self.desc[: h.numel()].copy_(h, non_blocking=True)
        size = [r.req.cells + r.req.cap_s + r.req.cap_w for r in models]
        self.h_order[slot].numpy()[:n] = np.argsort(-np.asarray(size), kind="stable")
        self.order[:n].copy_(self.h_order[slot][:n], non_blocking=True)
        b = self._batch(self.desc, n)
        n_team = sum(1 for r in models if self._team_model(r))
        t = abm.Tuning(self.block_threads, self.workgroups, self.items, self.team_size, n_team, 0,
                       0 if self.lds else 1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        abm._check(abm.lib().abm_predation_run_batched(C.byref(b), abm._p(self.order), 1 << 30,
                                                       C.byref(t), abm._p(self.ws),
                                                       self.ws.numel(), abm._stream()))
        e1.record(stream)
        self.h_out[slot][: n * self.desc_size].copy_(self.desc[: n * self.desc_size],
                                                     non_blocking=True)
        self.h_err[slot].copy_(self.ws[248:256], non_blocking=True)
        done = torch.cuda.Event()
        done.record(stream)
        return (slot, n, e0, e1, done)

    def collect(self, ticket):
        """Waits for a submitted chunk: (step, updates made in the chunk) per model."""
        abm = self.abm
        slot, n, e0, e1, done = ticket
        done.synchronize()
        self.busy_s += e0.elapsed_time(e1) / 1e3
        # the error word is sticky: non-zero once any team barrier or bounded
        # wait of this workspace has given up, which leaves the states invalid
        self.workspace_error = int(self.h_err[slot].view(self.torch.int64)[0].item())
        if self.workspace_error:
            raise RuntimeError("batched kernel: a team barrier gave up (workspace error word "
                               "set); the served states are not valid")
        raw = self.h_out[slot][: n * self.desc_size].numpy().tobytes()
        out = (abm.ModelDesc * n).from_buffer_copy(raw)
        return [(d.step, d.updates) for d in out]

    def finish(self, r: Running):
        """The model's last chunk is submitted.  With keep_results, its final
        state is read back now (waiting for that chunk), before a later chunk
        can reuse its ranges."""
        if not self.keep_results:
            return
        abm, torch = self.abm, self.torch
        q = r.req
        # a one-model view whose arrays start at this model's ranges
        d = self._descs([r], [r.step])
        d[0].cell_off = d[0].sheep_off = d[0].wolf_off = 0
        torch.cuda.synchronize()
        self.init_desc[: self.desc_size].copy_(self._stage(self.h_init[0], d, 1))
        cd = torch.zeros(q.cells, dtype=torch.int32, device=self.device)
        sp = lambda dd, o: abm.SpeciesPtrs(*(dd[k][o:].data_ptr() for k in ("x", "y", "e", "alive")))
        b = abm.Batch(1, self.max_cap, self.init_desc.data_ptr(), self.ready[r.cell_off:].data_ptr(),
                      self.claims[3 * r.cell_off:].data_ptr(), sp(self.sheep, r.sheep_off),
                      sp(self.wolves, r.wolf_off))
        abm._check(abm.lib().abm_predation_batched_grass(C.byref(b), abm._p(cd), abm._stream()))
        sheep = {k: v[r.sheep_off: r.sheep_off + q.cap_s].cpu().numpy()
                 for k, v in self.sheep.items()}
        wolves = {k: v[r.wolf_off: r.wolf_off + q.cap_w].cpu().numpy()
                  for k, v in self.wolves.items()}
        torch.cuda.synchronize()
        # the update count is complete once the scheduler has collected the chunk
        self.results[q.rid] = [cd.cpu().numpy(), sheep, wolves, r]

    def result(self, rid):
        """(grass countdowns, sheep, wolves, agent updates) of a finished model
        (keep_results), after the run."""
        cd, sheep, wolves, r = self.results[rid]
        return cd, sheep, wolves, r.updates


def requests_from_trace(trace) -> list:
    """workloads.served_trace() entries -> Request objects."""
    return [Request(i, t.arrival_s, t.side, t.steps, t.seed) for i, t in enumerate(trace)]
