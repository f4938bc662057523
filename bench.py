"""Benchmark of the select/update hot path on one MI355X.

Workload (one "step"): the select_update microbenchmark -- 2^24 agent slots x
8 int32 attributes in struct-of-arrays layout -- at the three mask densities
p in {0.001, 0.05, 0.5}.  For each density a step runs
  select_update  k = popcount(mask) distinct records into the selected slots,
  add_agents     k newborns into the free slots of alive = 1 - mask,
  remove_agents  kill mask = the same mask over the now all-live population
                 (which restores alive, so every step does identical work).
Ten seeded input sets (seeds 0-9) are resident in HBM and rotated step by step,
so the 256 MB last-level cache cannot hold a step's inputs from one use to
the next.  value = agent updates per second = (sum over densities of
3 * k) / (time per step).

Also printed: the HBM roofline of the dominant kernel (algorithmic bytes per
launch / mean launch time from HIP events on the launch stream) and the CPU
oracle timed on this host over a bounded sample.
"""
import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "agent-updates/s + %HBM peak, batched vs plain per-model launch; p99 latency"
N_SLOTS = 1 << 24
N_ATTRS = 8


LEGS = ("predation_small", "predation_large", "predation_large_multi_prey", "traffic", "lob",
        "sort_select", "batched", "batched_multi_prey", "table1_context")


def algorithmic_bytes(op, n, k):
    """Bytes the method must move per launch (see the roofline model)."""
    if op == "select_update":      # mask everywhere, k records read, k slots x 8 attrs written
        return n + 64 * k
    if op == "add_agents":         # alive everywhere, records read/written, alive set
        return 4 * n + 68 * k
    if op == "remove_agents":      # mask everywhere, alive read + written where killed
        return n + 8 * k
    raise ValueError(op)


def _profile_traffic(kernel_sources_hash, op):
    """HBM traffic per launch of `op` (mean over the densities) from the
    committed PMC summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "select_update_microbench_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"sources_sha256:\s*([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch\[" + op + r"\]:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_sources_hash:
        return None
    return float(t.group(1))


# The files the microbenchmark's kernels (select, add, remove) are built from.
MICROBENCH_SOURCES = ("include/abm.h", "paper_2508_16508_amd/csrc/api.hip",
                      "paper_2508_16508_amd/csrc/common.hpp", "paper_2508_16508_amd/csrc/scan.hpp",
                      "paper_2508_16508_amd/csrc/select.hip", "paper_2508_16508_amd/csrc/remove.hip",
                      "paper_2508_16508_amd/_build.py")


def kernel_sources_hash():
    """Hash of the microbenchmark kernels' sources and build flags: a counter
    summary taken on other sources no longer describes these kernels."""
    h = hashlib.sha256()
    for name in MICROBENCH_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _queue_ahead(torch):
    """Before a timed region that the host enqueues call by call: the device
    spins for about 100 ms, so the host has queued the region's launches by the
    time it starts and a host pause cannot leave the device idle inside the
    events; the collector stays off until the region is over (gc.enable)."""
    gc.disable()
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(250_000_000)


def _med(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def cpu_baseline(seeds=3, reps=5):
    """The oracle as it stands -- plain single-threaded C, built here with
    -O3 -march=native -- pinned to one core of this host.  Each call is timed
    alone (perf_counter around one C call on preallocated arrays: no input
    generation, no copies in the timed region); the median of `reps` calls
    per (seed, density, op).  The main figure is the microbenchmark step
    (select_update + add_agents + remove_agents at the three densities) on
    seeds 0..seeds-1, in agent updates per second like `value`."""
    import tempfile
    import oracle
    from oracle import build as obuild
    from paper_2508_16508_amd import workloads as W
    allowed = sorted(os.sched_getaffinity(0))
    info = {"cores": 1, "core_id": allowed[0], "nproc": len(allowed),
            "cpu_count": os.cpu_count(), "cpu_model": _cpu_model(),
            "build": "gcc -O3 -march=native (oracle/abm_oracle.c, built on this host)"}
    oracle.use_library(obuild.build_native(tempfile.mkdtemp(prefix="abm_oracle_")))
    os.sched_setaffinity(0, {allowed[0]})
    try:
        t_total, updates = 0.0, 0
        for seed in range(seeds):
            for p in W.DENSITIES:
                c = W.select_update_case(seed, p)
                out = c.attrs.copy()
                free = (1 - c.mask).astype(np.int32)
                ts = {"select": [], "add": [], "remove": []}
                for _ in range(reps):
                    t0 = time.perf_counter()
                    a, _ = oracle.select_update_into(out, c.mask, c.records)
                    ts["select"].append(time.perf_counter() - t0)
                    alive = free.copy()
                    t0 = time.perf_counter()
                    n_add, _ = oracle.add_agents_into(out, alive, c.records)
                    ts["add"].append(time.perf_counter() - t0)
                    t0 = time.perf_counter()
                    n_rem = oracle.remove_agents_into(alive, c.mask)
                    ts["remove"].append(time.perf_counter() - t0)
                assert a == n_add == n_rem == c.k
                t_total += sum(_med(v) for v in ts.values())
                updates += 3 * c.k
                del c, out, free, alive
        legs = cpu_baseline_legs(oracle, W)
    finally:
        os.sched_setaffinity(0, set(allowed))
    out = {"value": updates / t_total, "unit": "agent-updates/s", "kind": "oracle",
           "sample": f"seeds 0-{seeds - 1} of the 2^24 x 8 microbenchmark: select_update + "
                     f"add_agents + remove_agents at p in {{0.001, 0.05, 0.5}}, median of {reps} "
                     f"calls each ({t_total:.2f} s of oracle time per pass)",
           "legs": legs}
    out.update(info)
    return out


def _pred_leg(oracle, kw, steps, runs=1):
    """agent updates/s of the oracle on one predation model: `steps` steps
    from the initial state (init not timed), median over `runs` seeds."""
    rates = []
    for r in range(runs):
        P = oracle.pred_params(**dict(kw, seed=kw.get("seed", 0) + r))
        S = oracle.predation_init(P)
        t0 = time.perf_counter()
        st = oracle.predation_run(P, S, steps)
        dt = time.perf_counter() - t0
        rates.append(sum(s["live_s"] + s["live_w"] for s in st) / dt)
    return _med(rates)


def cpu_baseline_legs(oracle, W):
    """The pinned oracle on bounded samples of the other legs' workloads, in
    the same units as the GPU figures."""
    out = {}
    out["predation_small"] = {
        "value": _pred_leg(oracle, dict(seed=0), 200, runs=3), "unit": "agent-updates/s",
        "sample": "the 64x64 model (400 / 100 agents), 200 steps, seeds 0-2, median"}
    big = dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000, n_w0=400_000,
               seed=0)
    out["predation_large"] = {"value": _pred_leg(oracle, big, 10), "unit": "agent-updates/s",
                              "sample": "steps 0-9 of the 2048x2048 model, seed 0"}
    out["predation_large_multi_prey"] = {
        "value": _pred_leg(oracle, dict(big, multi_prey=1), 10), "unit": "agent-updates/s",
        "sample": "steps 0-9 of the 2048x2048 model with multi-prey, seed 0"}
    specs = W.batched_models(0, 4096)
    by_size = sorted(range(len(specs)), key=lambda m: specs[m].side)
    upd, dt = 0, 0.0
    for m in by_size[:: len(specs) // 32][:32]:
        sp = specs[m]
        P = oracle.pred_params(W=sp.side, H=sp.side, seed=sp.seed, cap_s=sp.cap_s,
                               cap_w=sp.cap_w, n_s0=sp.n_s0, n_w0=sp.n_w0)
        S = oracle.predation_init(P)
        t0 = time.perf_counter()
        upd += sum(s["live_s"] + s["live_w"] for s in oracle.predation_run(P, S, 20))
        dt += time.perf_counter() - t0
    out["batched"] = {"value": upd / dt, "unit": "agent-updates/s",
                      "sample": "32 models of the 4096-model batch (every 128th by size), "
                                "20 steps each, init not timed"}
    trace = W.served_trace(0)
    by_side = sorted(range(len(trace)), key=lambda i: trace[i].side)
    upd, dt = 0, 0.0
    for i in by_side[:: len(trace) // 24][:24]:
        q = trace[i]
        cells = q.side * q.side
        P = oracle.pred_params(W=q.side, H=q.side, seed=q.seed & 0xFFFFFFFF,
                               cap_s=max(1, 4 * (cells // 10)), cap_w=max(1, 4 * (cells // 40)),
                               n_s0=cells // 10, n_w0=cells // 40)
        S = oracle.predation_init(P)
        t0 = time.perf_counter()
        upd += sum(s["live_s"] + s["live_w"] for s in oracle.predation_run(P, S,
                                                                          min(q.steps, 20)))
        dt += time.perf_counter() - t0
    out["served"] = {"value": upd / dt, "unit": "agent-updates/s",
                     "sample": "24 requests of the served trace spread over its sides (every "
                               f"{len(trace) // 24}th by side), their first min(steps, 20) "
                               "steps each, init not timed"}
    upd, dt = 0, 0.0
    for r in range(3):
        P = oracle.traffic_params(100, seed=1 + r)
        S = oracle.traffic_init(P)
        oracle.traffic_run(P, S, 10)
        t0 = time.perf_counter()
        upd += sum(st["cars"] for st in oracle.traffic_run(P, S, 1000))
        dt += time.perf_counter() - t0
    out["traffic"] = {"value": upd / dt, "unit": "car-updates/s",
                      "sample": "roads 0-2, 1000 steps each after 10 warm-up steps"}
    dt = 0.0
    for bk in range(5):
        P = oracle.lob_params(cap=1000, traders=100, seed=1 + bk)
        S = oracle.lob_init(P)
        oracle.lob_run(P, S, 20)
        t0 = time.perf_counter()
        oracle.lob_run(P, S, 100)
        dt += time.perf_counter() - t0
    out["lob"] = {"value": 500 / dt, "unit": "book-steps/s",
                  "sample": "books 0-4, 100 steps each after 20 warm-up steps"}
    m = 1 << 22
    g = np.random.default_rng(7)
    key = g.integers(-2 ** 31, 2 ** 31, size=m, dtype=np.int64).astype(np.int32)
    attrs = W.int32_rows(8, 8, m)
    alive = np.ones(m, dtype=np.int32)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.sort_agents(attrs, key, alive=alive)
        ts.append(time.perf_counter() - t0)
    out["sort_agents"] = {"value": m / _med(ts), "unit": "agents/s",
                          "sample": "2^22 agents x 8 int32 + alive, full-range keys, median of 3 "
                                    "(the wrapper's input copies included)"}
    cond = W.bernoulli_mask(3, 0.05, 1 << 24)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.select_agents(cond)
        ts.append(time.perf_counter() - t0)
    out["select_agents"] = {"value": (1 << 24) / _med(ts), "unit": "agents/s",
                            "sample": "2^24 Bernoulli(0.05) flags, median of 3"}
    return out


def batched_leg(abm, W, torch, steps=500, chunk=50, plain_models=32, plain_steps=20, lds=True,
                max_side=256):
    """Batched form: 4096 uneven predation models (side 32-256, sheep = cells/10,
    wolves = cells/40, capacities 4x), `steps` steps as a graph of persistent
    launches of `chunk` steps each, against the one-model multi-launch path
    timed on a stratified subset of the same models (rates in agent updates/s;
    both paths compute bit-identical states).  max_side < 256 keeps only the
    models of at most that side (a profiling subset, not the workload)."""
    from paper_2508_16508_amd.tune import autotune_batched
    specs = [sp for sp in W.batched_models(0, 4096) if sp.side <= max_side]
    params = [abm.predation_params(W=sp.side, H=sp.side, seed=sp.seed, cap_s=sp.cap_s,
                                   cap_w=sp.cap_w, n_s0=sp.n_s0, n_w0=sp.n_w0) for sp in specs]
    def make(block, items):
        b = abm.BatchedPredation(params, 1000, block_threads=block, items=items, lds=lds)
        b.init()
        return b

    # tuned on the batch itself (occupancy depends on how many models compete)
    tuning = autotune_batched(make, "batched:4096 models side 32-256", steps=4, use_cache=False)
    torch.cuda.empty_cache()
    batch = abm.BatchedPredation(params, steps, block_threads=tuning["block_threads"],
                                 items=tuning["items"], lds=lds)
    lds_models, lds_cells = batch.lds_models(), batch.lds_cells()
    batch.init()
    batch.run(1)                           # warm-up (first step of every model)
    # the rest of the rollout, captured once by the library as a graph of
    # persistent launches of `chunk` steps
    graph = batch.capture(chunk, (steps - 1 + chunk - 1) // chunk)
    torch.cuda.synchronize()
    d0 = batch.descriptors()
    u0 = sum(d.updates for d in d0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d1 = batch.descriptors()
    assert all(d.step == steps for d in d1)
    updates = sum(d.updates for d in d1) - u0
    err = abm.workspace_error(batch.ws)
    cells = sum(sp.side * sp.side for sp in specs)
    graph.destroy()
    del batch, graph
    torch.cuda.empty_cache()

    # one-model path on a stratified subset (every 128th model by size)
    by_size = sorted(range(len(specs)), key=lambda m: specs[m].side)
    pick = by_size[:: max(1, len(specs) // plain_models)][:plain_models]
    models = [abm.predation_init(params[m]) for m in pick]
    stats = [torch.zeros((plain_steps, 8), dtype=torch.int64, device="cuda") for _ in pick]
    for mdl in models:
        mdl.run(1)                          # warm-up
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record()
    for mdl, st in zip(models, stats):
        mdl.run(plain_steps, st)
    p1.record()
    torch.cuda.synchronize()
    pms = p0.elapsed_time(p1)
    pupd = sum(int(st[:, 0].sum().item() + st[:, 1].sum().item()) for st in stats)
    rate_b = updates / (ms / 1e3)
    rate_p = pupd / (pms / 1e3)
    subset = "" if max_side >= 256 else f" (only the {len(specs)} of side <= {max_side})"
    return {"workload": "4096 predation models, side uniform in [32, 256], sheep = cells/10, "
                        f"wolves = cells/40, capacities 4x, seeds base+m{subset}; "
                        f"{steps - 1} timed steps as one library-captured graph of {chunk}-step "
                        "persistent launches",
            "cells": cells, "agent_updates": updates, "ms": ms,
            "agent_updates_per_s": rate_b,
            "plain_agent_updates_per_s": rate_p,
            "plain_sample": f"{len(pick)} models (every {len(specs) // plain_models}th by size), "
                            f"{plain_steps} steps each, one-model multi-launch path",
            "batched_over_plain": rate_b / rate_p,
            "workspace_error": err,
            "lds_claim_models": lds_models,
            "lds_claim_max_cells": lds_cells,
            "tuning": {"block_threads": tuning["block_threads"], "items": tuning["items"],
                       "candidates_ms_per_4_steps": tuning["timings_ms"]}}


def table1_context_leg(abm, torch, runs=10):
    """The paper's Table 1 shapes with the small model's parameters: 100 x 100
    with 600 sheep + 400 wolves and 1000 x 1000 with 6000 + 4000 (capacities
    ten times the initial agents), on the one-model path and as the only model
    of the batched form; 100 steps timed as the paper times them, the median
    over `runs` fresh models of 105 steps less the median of 5 steps (device
    events around each run).  Context only: the paper's figures come from other
    hardware and software."""
    out = {"method": "median(105 steps) - median(5 steps) over %d fresh models" % runs}
    for name, side, ns, nw in (("small", 100, 600, 400), ("large", 1000, 6000, 4000)):
        kw = dict(W=side, H=side, seed=0, cap_s=10 * ns, cap_w=10 * nw, n_s0=ns, n_w0=nw)
        res = {}
        for path in ("one_model", "batched"):
            med = {}
            for steps in (105, 5):
                ts = []
                for r in range(runs):
                    p = abm.predation_params(**dict(kw, seed=r))
                    if path == "one_model":
                        m = abm.predation_init(p)
                        run = lambda: m.run(steps)
                    else:
                        m = abm.BatchedPredation([p], steps, block_threads=1024, items=2)
                        m.init()
                        run = lambda: m.run(steps)
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    run()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1))
                    del m
                med[steps] = _med(ts)
            res[path + "_ms_per_100_steps"] = med[105] - med[5]
        out[name] = dict(workload=f"{side}x{side}, {ns} sheep + {nw} wolves, 100 steps", **res)
    out["paper_abmax_rm_ms"] = {"small": 50.26, "large": 3315.88}
    return out


def predation_leg(abm, torch, kw, steps, label):
    """One model on the one-model path (three launches per step): agent updates
    per second over `steps` steps (live agents at the start of each step)."""
    model = abm.predation_init(abm.predation_params(**kw))
    stats = torch.zeros((steps, 8), dtype=torch.int64, device="cuda")
    model.run(1)                                   # warm-up step
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    _queue_ahead(torch)
    e0.record()
    model.run(steps, stats)
    e1.record()
    torch.cuda.synchronize()
    gc.enable()
    ms = e0.elapsed_time(e1)
    upd = int(stats[:, 0].sum().item() + stats[:, 1].sum().item())
    err = abm.workspace_error(model.ws)
    del model, stats
    torch.cuda.empty_cache()
    return {"workload": label, "steps": steps, "ms": ms, "us_per_step": 1e3 * ms / steps,
            "agent_updates": upd, "agent_updates_per_s": upd / (ms / 1e3),
            "workspace_error": err}


def sort_select_leg(abm, torch, W, n=1 << 24, reps=5):
    """sort_agents on the microbenchmark's collection (2^24 agents x 8 int32
    attributes + alive, full-range random int32 keys; radix sort plus the
    gather of 9 columns) and select_agents (stable partition) at p = 0.05."""
    import numpy as np
    dev = torch.device("cuda")
    g = np.random.default_rng(7)
    key = torch.from_numpy(g.integers(-2 ** 31, 2 ** 31, size=n, dtype=np.int64)
                           .astype(np.int32)).to(dev)
    attrs = torch.from_numpy(W.int32_rows(8, 8, n)).to(dev)
    alive = torch.ones(n, dtype=torch.int32, device=dev)
    cond = torch.from_numpy(W.bernoulli_mask(3, 0.05, n)).to(dev)
    ws = abm.sort_workspace(n, dev, n_cols=9)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out = {}
    for name, fn in (("sort_agents", lambda: abm.sort_agents(attrs, key, alive=alive, perm=perm,
                                                              ws=ws)),
                     ("select_agents", lambda: abm.select_agents(cond, order=order, ws=ws,
                                                                  count=count))):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "agents_per_s": n / (ms / 1e3)}
    out["workload"] = ("2^24 agents x 8 int32 attributes + alive, full-range random int32 keys "
                       "(sort), Bernoulli(0.05) condition (select); mean of 5 calls")
    del key, attrs, alive, cond, ws, perm, order
    torch.cuda.empty_cache()
    return out


def lob_leg(abm, torch, n_books=500, cap=1000, traders=100, steps=100):
    """Limit order books (Sec. 5.3): n_books books of `cap` order slots with
    `traders` noisy traders each, `steps` steps in one call (one workgroup per
    book, the book in LDS, all books matched at once)."""
    books = abm.OrderBooks(abm.lob_params(cap=cap, traders=traders, seed=1), n_books)
    books.init()
    books.run(20)                                  # warm-up: the books fill
    stats = torch.zeros((steps, n_books, 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    books.run(steps, stats)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    orders = int((stats[:, :, 0] + stats[:, :, 1]).sum().item())
    volume = int(stats[:, :, 5].sum().item())
    del books, stats
    return {"workload": f"{n_books} books of {cap} slots, {traders} traders each, {steps} steps "
                        "in one call, orders with probability 1/2, spread 20 ticks, qty 1-10, "
                        "expiry 20 steps", "steps": steps, "ms": ms,
            "resting_orders_per_step": orders / steps, "shares_matched": volume,
            "book_steps_per_s": n_books * steps / (ms / 1e3)}


def batched_multi_prey_leg(abm, W, torch, steps=200, chunk=50, block=512, items=2):
    """The 4096-model batch of the batched leg with multi-prey (the wolves and
    sheep of a cell paired by rank) in every model, run as `steps` launches of
    `chunk` steps at one fixed shape after a warm-up step, against the same
    batch with the one-prey rule at that shape."""
    specs = W.batched_models(0, 4096)
    out = {"workload": "4096 predation models as in the batched leg, multi-prey in every model; "
                       f"{steps} timed steps as {steps // chunk} persistent launches of {chunk} "
                       f"steps, {block} threads x {items} items",
           "block_threads": block, "items": items}
    for multi in (1, 0):
        params = [abm.predation_params(W=sp.side, H=sp.side, seed=sp.seed, cap_s=sp.cap_s,
                                       cap_w=sp.cap_w, n_s0=sp.n_s0, n_w0=sp.n_w0,
                                       multi_prey=multi) for sp in specs]
        b = abm.BatchedPredation(params, steps + 1, block_threads=block, items=items)
        b.init()
        b.run(1)
        torch.cuda.synchronize()
        u0 = sum(d.updates for d in b.descriptors())
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps // chunk):
            b.run(chunk)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        d1 = b.descriptors()
        assert all(d.step == steps + 1 for d in d1)
        rate = (sum(d.updates for d in d1) - u0) / (ms / 1e3)
        err = abm.workspace_error(b.ws)
        if multi:
            out.update(ms=ms, agent_updates_per_s=rate, workspace_error=err)
        else:
            out.update(one_prey_ms=ms, one_prey_agent_updates_per_s=rate)
            out["workspace_error"] = max(out["workspace_error"], err)
        del b
        torch.cuda.empty_cache()
    return out


def traffic_leg(abm, torch, n_roads=500, length=100, steps=1000):
    """Traffic CA (Sec. 5.2): n_roads roads of 3 x length cells, `steps` steps in
    one call (one workgroup per road, the road held in LDS); car updates per
    second = cars at the start of each step, summed over roads and steps."""
    roads = abm.TrafficRoads(abm.traffic_params(length, seed=1), n_roads)
    roads.init()
    roads.run(10)                                  # warm-up: the roads fill up
    stats = torch.zeros((steps, n_roads, 8), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    roads.run(steps, stats)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    cars = int(stats[:, :, 0].sum().item())
    del roads, stats
    return {"workload": f"{n_roads} roads of 3 x {length} cells, {steps} steps in one call, "
                        "lights and spawns with probability 1/2, seeds 1..", "steps": steps,
            "ms": ms, "car_updates": cars, "car_updates_per_s": cars / (ms / 1e3)}


def served_leg(seconds, rate=200.0, team_size=4, team_min_size=1 << 18, depth=1,
               budget=1 << 23):
    """Served form: Poisson arrivals (rate/s for `seconds`), grid side log-uniform
    in [32, 1024], steps log-uniform in [100, 5000], admitted by HBM footprint
    into the running batched launch; open-loop latency from scheduled arrival.
    With team_size > 1, models of at least team_min_size cells plus slots
    (side >= ~400) are each advanced by a team of team_size workgroups, and the
    scheduler gives such a model team_size times the step budget of a solo one.
    Under this load teams of 4 halve the p99 latency of teams of 1 and raise
    throughput by a third; 8 is slightly faster with a longer tail, 16 too coarse.
    depth = chunks in flight: 2 plans and submits the next chunk while one
    runs; measured, the device was already busy 99.4 % of the time with 1, so
    2 left the rate unchanged and raised the median latency (a new request
    then waits behind two chunks)."""
    from paper_2508_16508_amd import serve as S
    from paper_2508_16508_amd import workloads as W
    trace = W.served_trace(0, rate=rate, duration_s=seconds)
    reqs = S.requests_from_trace(trace)
    cells, sheep, wolves = 400_000_000, 160_000_000, 40_000_000
    runner = S.GpuRunner(cells, sheep, wolves,
                         max_model_cap=max(max(q.cap_s, q.cap_w) for q in reqs),
                         team_size=team_size, team_min_size=team_min_size)
    sch = S.Scheduler(runner, cells, sheep, wolves, slot_step_budget=budget, depth=depth,
                      log=lambda m: print("served:", m, file=sys.stderr, flush=True))
    rep = sch.serve(reqs)
    out = rep.summary()
    out["workspace_error"] = runner.workspace_error
    out["workload"] = (f"Poisson arrivals at {rate:g}/s for {seconds:g} s ({len(reqs)} requests), "
                       "side log-uniform [32, 1024], steps log-uniform [100, 5000], "
                       "sheep = cells/10, wolves = cells/40, capacities 4x")
    out["pools"] = {"cells": cells, "sheep_slots": sheep, "wolf_slots": wolves}
    out["teams"] = {"team_size": team_size, "team_min_size": team_min_size}
    out["chunks_in_flight"], out["slot_step_budget"] = depth, budget
    # every request completes, so the work is fixed by the trace: the served
    # rate cannot exceed the work over the trace's duration
    out["offered_agent_updates_per_s"] = out["agent_updates"] / seconds
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sets", type=int, default=10, help="rotated input sets (seeds 0..sets-1)")
    ap.add_argument("--cpu-seeds", type=int, default=3,
                    help="microbenchmark seeds timed in the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="run none of the legs below")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run after the microbenchmark")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device-to-device 3 times (a transfer of known size "
                         "for scaling hardware byte counters)")
    ap.add_argument("--batched-lds", choices=("on", "off"), default="on",
                    help="keep the claim tables of the batch's smallest models in LDS")
    ap.add_argument("--batched-max-side", type=int, default=256,
                    help="profiling: keep only the batch's models of at most this side")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the served request trace (0 = skip)")
    ap.add_argument("--served-team-size", type=int, default=4,
                    help="workgroups per team for the large models of the served leg (1 = none)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2508_16508_amd as abm
    from paper_2508_16508_amd import workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---- resident inputs: per seed and density, mask + records + alive
    sets = []
    for seed in range(args.sets):
        per_p = []
        for p in W.DENSITIES:
            c = W.select_update_case(seed, p, with_attrs=False)
            mask = torch.from_numpy(c.mask).to(dev)
            per_p.append(dict(p=p, k=c.k, mask=mask, rec=torch.from_numpy(c.records).to(dev),
                              alive=(1 - mask).to(torch.int32)))
        sets.append(per_p)
    dst = torch.zeros((N_ATTRS, N_SLOTS), dtype=torch.int32, device=dev)
    ws = abm.workspace(N_SLOTS, abm.ABM_OP_SELECT_UPDATE, dev)
    cnt = torch.zeros(8, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    ops = ("select_update", "add_agents", "remove_agents")
    events = {op: [] for op in ops}

    def step(s, timed):
        for d in sets[s % len(sets)]:
            for op in ops:
                if timed:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                if op == "select_update":
                    abm.select_update(dst, d["mask"], d["rec"], ws=ws, applied=cnt[0:1],
                                      dropped=cnt[1:2])
                elif op == "add_agents":
                    abm.add_agents(dst, d["alive"], d["rec"], ws=ws, added=cnt[2:3],
                                   dropped=cnt[3:4])
                else:
                    abm.remove_agents(d["alive"], d["mask"], ws=ws, removed=cnt[4:5])
                if timed:
                    e1.record(stream)
                    events[op].append((e0, e1, d["k"], d["p"]))

    # every resident input set is used once before the warm-up steps (the
    # timed steps rotate over all of them: no first use falls in the timed
    # region), then the W warm-up steps
    for s in range(len(sets)):
        step(s, False)
    for s in range(args.warmup):
        step(s, False)
    torch.cuda.synchronize()
    # the device starts the timed launches only after a spin long enough for
    # the host to queue all of them, so the events time the device and not
    # the host: a host pause inside a call (a fresh box's first process has
    # shown 40 ms ones) would otherwise leave the device idle inside that
    # launch's events; the collector stays off while the calls are made
    _queue_ahead(torch)
    t0 = time.perf_counter()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for s in range(args.steps):
        step(args.warmup + s, True)
    g1.record(stream)
    torch.cuda.synchronize()
    gc.enable()
    wall = time.perf_counter() - t0
    ms_total = g0.elapsed_time(g1)
    ms_per_step = ms_total / args.steps

    # the kernels' give-up word: set if a bounded wait of the single-pass scan
    # ever expired (its ordering assumption failed), which would make the
    # timed state wrong
    micro_err = abm.workspace_error(ws)
    # correctness of the timed work: the last density's counts and restored alive
    last = sets[(args.warmup + args.steps - 1) % len(sets)][-1]
    c = cnt.cpu().numpy()
    assert c[0] == last["k"] and c[1] == 0 and c[2] == last["k"] and c[4] == last["k"], c
    assert int((last["alive"] == 0).sum().item()) == last["k"]

    updates = 0
    for s in range(args.steps):
        updates += sum(3 * d["k"] for d in sets[(args.warmup + s) % len(sets)])
    value = updates / (ms_total / 1e3)

    kernels = {}
    for op in ops:
        durs = [e0.elapsed_time(e1) * 1e-3 for e0, e1, _, _ in events[op]]
        byts = [algorithmic_bytes(op, N_SLOTS, k) for _, _, k, _ in events[op]]
        mean_s = float(np.mean(durs))
        by_p = {}
        for p in W.DENSITIES:
            dp = [e0.elapsed_time(e1) * 1e-3 for e0, e1, _, pp in events[op] if pp == p]
            bp = [algorithmic_bytes(op, N_SLOTS, k) for _, _, k, pp in events[op] if pp == p]
            by_p[str(p)] = dict(mean_us=float(np.mean(dp)) * 1e6,
                                gbs=float(np.mean(bp)) / float(np.mean(dp)) / 1e9)
        kernels[op] = dict(launches=len(durs), mean_us=mean_s * 1e6, total_ms=sum(durs) * 1e3,
                           bytes_per_launch=float(np.mean(byts)),
                           gbs=float(np.mean(byts)) / mean_s / 1e9, by_density=by_p)
    dom = max(ops, key=lambda o: kernels[o]["total_ms"])
    kd = kernels[dom]
    src_hash = kernel_sources_hash()
    traffic = _profile_traffic(src_hash, dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kd["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": kd["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": kd["bytes_per_launch"],
                "mean_launch_us": kd["mean_us"]}

    out = {
        "metric": METRIC, "value": value, "unit": "agent-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "select_update microbench (2^24 slots x 8 int32 SoA; "
                               "select_update + add_agents + remove_agents at p in "
                               "{0.001, 0.05, 0.5}; seeds 0-9 resident and rotated)",
                   "slots": N_SLOTS, "attrs": N_ATTRS, "densities": list(W.DENSITIES),
                   "input_sets": args.sets, "wall_s": wall},
        "roofline": roofline,
        "kernels": kernels,
        "kernel_sources": src_hash,
        "workspace_error": {"microbench": micro_err},
    }
    del sets, dst
    torch.cuda.empty_cache()
    legs = [] if args.no_batched else args.legs.split(",")
    unknown = set(legs) - set(LEGS)
    if unknown:
        raise SystemExit(f"unknown legs {sorted(unknown)}; known: {', '.join(LEGS)}")
    if "predation_small" in legs:
        out["predation_small"] = predation_leg(
            abm, torch, dict(seed=0), 199,
            "64x64 torus, 400 sheep / 100 wolves in 4096 / 1024 slots, steps 1-199 after a "
            "warm-up step")
    if "predation_large" in legs:
        out["predation_large"] = predation_leg(
            abm, torch, dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000,
                             n_w0=400_000, seed=0), 999,
            "2048x2048 torus, 1.6M sheep / 0.4M wolves in 2^24 / 2^22 slots, steps 1-999 "
            "after a warm-up step")
    if "predation_large_multi_prey" in legs:
        out["predation_large_multi_prey"] = predation_leg(
            abm, torch, dict(W=2048, H=2048, cap_s=1 << 24, cap_w=1 << 22, n_s0=1_600_000,
                             n_w0=400_000, seed=0, multi_prey=1), 999,
            "2048x2048 torus as above with prey matched by rank within each cell (the r-th "
            "wolf of a cell eats its r-th sheep), steps 1-999 after a warm-up step")
    if "traffic" in legs:
        out["traffic"] = traffic_leg(abm, torch)
    if "lob" in legs:
        out["lob"] = lob_leg(abm, torch)
    if "sort_select" in legs:
        out["sort_select"] = sort_select_leg(abm, torch, W)
    if "batched" in legs:
        out["batched"] = batched_leg(abm, W, torch, lds=args.batched_lds == "on",
                                     max_side=args.batched_max_side)
    if "batched_multi_prey" in legs:
        out["batched_multi_prey"] = batched_multi_prey_leg(abm, W, torch)
    if "table1_context" in legs:
        out["table1_context"] = table1_context_leg(abm, torch)
    torch.cuda.empty_cache()
    if args.served_seconds > 0:
        out["served"] = served_leg(args.served_seconds, team_size=args.served_team_size)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seeds)
    for leg in ("predation_small", "predation_large", "predation_large_multi_prey", "batched",
                "batched_multi_prey", "served"):
        if leg in out:
            out["workspace_error"][leg] = out[leg]["workspace_error"]
    print(json.dumps(out), flush=True)
    bad = {k: v for k, v in out["workspace_error"].items() if v}
    if bad:
        print(f"bench.py: a kernel's bounded wait gave up in {sorted(bad)}: the timed state is "
              "not valid", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
