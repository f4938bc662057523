"""CPU oracle for the ABMax select/update hot path (arXiv 2508.16508).

TEST INFRASTRUCTURE ONLY.  This package wraps ``liboracle.so`` (built from
``abm_oracle.c`` by :func:`oracle.build.build`) with ctypes and numpy.  Only the
test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product library never does.  It shares no code
with the HIP path.

Every function here is a thin marshalling layer: the arithmetic lives in the C
file, written as plain sequential definitions (Sec. 4 toy task, Alg. 1/2,
Sec. 2 API list, Sec. 5.1 predation model).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def use_library(path: str):
    """Bind this module to another build of the same source (the timing build
    of build.build_native); must come before any other call in the process."""
    global _lib, LIB_PATH
    if _lib is not None and LIB_PATH != path:
        raise RuntimeError("the oracle library is already loaded from " + LIB_PATH)
    LIB_PATH = path


def lib():
    """Load liboracle.so, building it first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class PredParams(C.Structure):
    """Predation model parameters (Sec. 5.1; the values are not given in the
    paper and are fixed by the workload definition)."""
    _fields_ = [
        ("W", C.c_int32), ("H", C.c_int32), ("R", C.c_int32),
        ("gain_s", C.c_int32), ("gain_w", C.c_int32),
        ("T_s", C.c_uint32), ("T_w", C.c_uint32), ("seed", C.c_uint32),
        ("cap_s", C.c_int64), ("cap_w", C.c_int64),
        ("n_s0", C.c_int64), ("n_w0", C.c_int64),
        ("multi_prey", C.c_int32),
    ]


class _Species(C.Structure):
    _fields_ = [("x", C.POINTER(C.c_int32)), ("y", C.POINTER(C.c_int32)),
                ("e", C.POINTER(C.c_int32)), ("alive", C.POINTER(C.c_int32))]


class _PredState(C.Structure):
    _fields_ = [("grass", C.POINTER(C.c_int32)), ("sheep", _Species),
                ("wolves", _Species), ("step", C.c_uint32)]


class PredStats(C.Structure):
    _fields_ = [("live_s", C.c_int64), ("live_w", C.c_int64),
                ("grass_eaten", C.c_int64), ("sheep_eaten", C.c_int64),
                ("births_s", C.c_int64), ("births_w", C.c_int64),
                ("starved_s", C.c_int64), ("starved_w", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class LobParams(C.Structure):
    """Limit order book parameters (Sec. 5.3; the paper gives no values)."""
    _fields_ = [("cap", C.c_int32), ("traders", C.c_int32), ("T_order", C.c_uint32),
                ("spread", C.c_int32), ("max_qty", C.c_int32), ("expiry", C.c_int32),
                ("price0", C.c_int32), ("seed", C.c_uint32)]


class _LobState(C.Structure):
    _fields_ = [("side", C.POINTER(C.c_int32)), ("price", C.POINTER(C.c_int32)),
                ("qty", C.POINTER(C.c_int32)), ("time", C.POINTER(C.c_int32)),
                ("alive", C.POINTER(C.c_int32)), ("last_price", C.c_int32),
                ("step", C.c_uint32)]


class LobStats(C.Structure):
    _fields_ = [("buys", C.c_int64), ("sells", C.c_int64), ("placed", C.c_int64),
                ("dropped", C.c_int64), ("expired", C.c_int64), ("volume", C.c_int64),
                ("filled_orders", C.c_int64), ("price", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TrafficParams(C.Structure):
    """Traffic CA parameters (Sec. 5.2; the paper gives no values)."""
    _fields_ = [("length", C.c_int32), ("T_green", C.c_uint32), ("T_spawn", C.c_uint32),
                ("seed", C.c_uint32)]


class _TrafficState(C.Structure):
    _fields_ = [("lane", C.POINTER(C.c_int32)), ("pos", C.POINTER(C.c_int32)),
                ("alive", C.POINTER(C.c_int32)), ("step", C.c_uint32)]


class TrafficStats(C.Structure):
    _fields_ = [("cars", C.c_int64), ("exited", C.c_int64), ("moved", C.c_int64),
                ("blocked", C.c_int64), ("lost", C.c_int64), ("waiting_red", C.c_int64),
                ("spawned", C.c_int64), ("lane_changes", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_P8 = C.POINTER(C.c_uint8)
_P32 = C.POINTER(C.c_int32)
_PU32 = C.POINTER(C.c_uint32)
_P64 = C.POINTER(C.c_int64)
_PU64 = C.POINTER(C.c_uint64)
_PP32 = C.POINTER(C.POINTER(C.c_int32))


def _declare(L):
    L.orc_mix64.argtypes = [C.c_uint64]
    L.orc_mix64.restype = C.c_uint64
    L.orc_rng.argtypes = [C.c_uint32] * 4
    L.orc_rng.restype = C.c_uint32
    L.orc_uniform.argtypes = [C.c_uint32, C.c_uint32]
    L.orc_uniform.restype = C.c_uint32
    L.orc_toy_rank_match.argtypes = [_P64, C.c_int64, _P64, C.c_int64, C.c_int, _P64]
    L.orc_toy_rank_match.restype = None
    L.orc_toy_sort_count_iterate.argtypes = [_P64, C.c_int64, _P64, C.c_int64, _P64]
    L.orc_toy_sort_count_iterate.restype = None
    L.orc_select_indices.argtypes = [_P8, C.c_int64, _P64]
    L.orc_select_indices.restype = C.c_int64
    L.orc_select_update.argtypes = [C.c_int64, C.c_int32, _PP32, _P8, C.c_int64, _PP32, _P8,
                                    _P64, _P64]
    L.orc_select_update.restype = None
    L.orc_add_agents.argtypes = [C.c_int64, C.c_int32, _PP32, _P32, C.c_int64, _PP32, _P64, _P64]
    L.orc_add_agents.restype = None
    L.orc_remove_agents.argtypes = [C.c_int64, _P32, _P8, _P64]
    L.orc_remove_agents.restype = None
    L.orc_resolve_conflicts.argtypes = [C.c_int64, _P32, _PU32, _P8, C.c_int64, _PU64, _P32, _P8]
    L.orc_resolve_conflicts.restype = None
    L.orc_predation_init.argtypes = [C.POINTER(PredParams), C.POINTER(_PredState)]
    L.orc_predation_init.restype = None
    L.orc_predation_step.argtypes = [C.POINTER(PredParams), C.POINTER(_PredState),
                                     C.POINTER(PredStats)]
    L.orc_predation_step.restype = None
    L.orc_sort_agents.argtypes = [C.c_int64, C.c_int32, _PP32, _P32, _P32, C.c_int32, _P32]
    L.orc_sort_agents.restype = None
    L.orc_select_agents.argtypes = [_P8, C.c_int64, _P32]
    L.orc_select_agents.restype = C.c_int64
    L.orc_lob_init.argtypes = [C.POINTER(LobParams), C.POINTER(_LobState)]
    L.orc_lob_init.restype = None
    L.orc_lob_step.argtypes = [C.POINTER(LobParams), C.POINTER(_LobState), C.POINTER(LobStats)]
    L.orc_lob_step.restype = None
    L.orc_traffic_init.argtypes = [C.POINTER(TrafficParams), C.POINTER(_TrafficState)]
    L.orc_traffic_init.restype = None
    L.orc_traffic_step.argtypes = [C.POINTER(TrafficParams), C.POINTER(_TrafficState),
                                   C.POINTER(TrafficStats)]
    L.orc_traffic_step.restype = None


def _ptr(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(ct))


def _ptr_array(rows: np.ndarray):
    """An array of row pointers for a C-contiguous 2-D int32 array."""
    assert rows.dtype == np.int32 and rows.ndim == 2 and rows.flags["C_CONTIGUOUS"]
    arr = (C.POINTER(C.c_int32) * max(1, rows.shape[0]))()
    for a in range(rows.shape[0]):
        arr[a] = rows[a].ctypes.data_as(C.POINTER(C.c_int32))
    return arr


# ---------------------------------------------------------------- RNG

def mix64(z: int) -> int:
    return int(lib().orc_mix64(z & 0xFFFFFFFFFFFFFFFF))


def rng(seed: int, step: int, agent: int, purpose: int) -> int:
    return int(lib().orc_rng(seed & 0xFFFFFFFF, step & 0xFFFFFFFF, agent & 0xFFFFFFFF,
                             purpose & 0xFFFFFFFF))


def uniform(h: int, n: int) -> int:
    return int(lib().orc_uniform(h, n))


# ---------------------------------------------------------------- toy task

def toy_rank_match(a, b, guard: bool = True) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    out = np.empty(max(1, a.size), dtype=np.int64)
    lib().orc_toy_rank_match(_ptr(a, C.c_int64), a.size, _ptr(b, C.c_int64), b.size,
                             int(guard), _ptr(out, C.c_int64))
    return out[: a.size]


def toy_sort_count_iterate(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    out = np.empty(max(1, a.size), dtype=np.int64)
    lib().orc_toy_sort_count_iterate(_ptr(a, C.c_int64), a.size, _ptr(b, C.c_int64), b.size,
                                     _ptr(out, C.c_int64))
    return out[: a.size]


# ---------------------------------------------------------------- primitives

def select_indices(mask) -> np.ndarray:
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.empty(max(1, mask.size), dtype=np.int64)
    k = lib().orc_select_indices(_ptr(mask, C.c_uint8), mask.size, _ptr(out, C.c_int64))
    return out[:k].copy()


def select_update(attrs, sel_mask, recs, upd_mask=None):
    """Returns (new_attrs [A, n], applied, dropped).  attrs is not modified."""
    out = np.array(attrs, dtype=np.int32, order="C", copy=True)
    recs = np.ascontiguousarray(recs, dtype=np.int32)
    sel_mask = np.ascontiguousarray(sel_mask, dtype=np.uint8)
    assert out.ndim == 2 and recs.ndim == 2 and recs.shape[0] == out.shape[0]
    assert sel_mask.size == out.shape[1]
    um = None
    if upd_mask is not None:
        upd_mask = np.ascontiguousarray(upd_mask, dtype=np.uint8)
        assert upd_mask.size == recs.shape[1]
        um = _ptr(upd_mask, C.c_uint8)
    applied, dropped = C.c_int64(), C.c_int64()
    pa, pr = _ptr_array(out), _ptr_array(recs)
    lib().orc_select_update(out.shape[1], out.shape[0], pa, _ptr(sel_mask, C.c_uint8),
                            recs.shape[1], pr, um, C.byref(applied), C.byref(dropped))
    return out, applied.value, dropped.value


def select_update_into(out, sel_mask, recs):
    """select_update applied in place to the C-contiguous int32 [A, n] array
    `out` (no copies; for timing).  Returns (applied, dropped)."""
    assert out.dtype == np.int32 and out.flags["C_CONTIGUOUS"]
    applied, dropped = C.c_int64(), C.c_int64()
    lib().orc_select_update(out.shape[1], out.shape[0], _ptr_array(out),
                            _ptr(sel_mask, C.c_uint8), recs.shape[1], _ptr_array(recs), None,
                            C.byref(applied), C.byref(dropped))
    return applied.value, dropped.value


def add_agents_into(out, alive, recs):
    """add_agents applied in place to `out` and `alive` (no copies; for
    timing).  Returns (added, dropped)."""
    assert out.dtype == np.int32 and out.flags["C_CONTIGUOUS"] and alive.flags["C_CONTIGUOUS"]
    added, dropped = C.c_int64(), C.c_int64()
    lib().orc_add_agents(out.shape[1], out.shape[0], _ptr_array(out), _ptr(alive, C.c_int32),
                         recs.shape[1], _ptr_array(recs), C.byref(added), C.byref(dropped))
    return added.value, dropped.value


def remove_agents_into(alive, kill):
    """remove_agents applied in place to `alive` (no copies; for timing)."""
    assert alive.dtype == np.int32 and alive.flags["C_CONTIGUOUS"]
    removed = C.c_int64()
    lib().orc_remove_agents(alive.size, _ptr(alive, C.c_int32), _ptr(kill, C.c_uint8),
                            C.byref(removed))
    return removed.value


def add_agents(attrs, alive, recs):
    """Returns (new_attrs, new_alive, added, dropped)."""
    out = np.array(attrs, dtype=np.int32, order="C", copy=True)
    al = np.array(alive, dtype=np.int32, copy=True)
    recs = np.ascontiguousarray(recs, dtype=np.int32)
    assert recs.shape[0] == out.shape[0] and al.size == out.shape[1]
    added, dropped = C.c_int64(), C.c_int64()
    pa, pr = _ptr_array(out), _ptr_array(recs)
    lib().orc_add_agents(out.shape[1], out.shape[0], pa, _ptr(al, C.c_int32), recs.shape[1], pr,
                         C.byref(added), C.byref(dropped))
    return out, al, added.value, dropped.value


def remove_agents(alive, kill):
    """Returns (new_alive, removed)."""
    al = np.array(alive, dtype=np.int32, copy=True)
    kill = np.ascontiguousarray(kill, dtype=np.uint8)
    assert kill.size == al.size
    removed = C.c_int64()
    lib().orc_remove_agents(al.size, _ptr(al, C.c_int32), _ptr(kill, C.c_uint8),
                            C.byref(removed))
    return al, removed.value


def resolve_conflicts(target, prio, n_targets, active=None):
    """Returns (best uint64[n_targets], winner int32[n_targets], won uint8[n_claims])."""
    target = np.ascontiguousarray(target, dtype=np.int32)
    prio = np.ascontiguousarray(prio, dtype=np.uint32)
    n = target.size
    assert prio.size == n
    act = None
    if active is not None:
        active = np.ascontiguousarray(active, dtype=np.uint8)
        assert active.size == n
        act = _ptr(active, C.c_uint8)
    best = np.empty(max(1, n_targets), dtype=np.uint64)
    winner = np.empty(max(1, n_targets), dtype=np.int32)
    won = np.empty(max(1, n), dtype=np.uint8)
    lib().orc_resolve_conflicts(n, _ptr(target, C.c_int32), _ptr(prio, C.c_uint32), act,
                                n_targets, _ptr(best, C.c_uint64), _ptr(winner, C.c_int32),
                                _ptr(won, C.c_uint8))
    return best[:n_targets].copy(), winner[:n_targets].copy(), won[:n].copy()


# ---------------------------------------------------------------- predation

# Workload parameters of the small predation model: 64x64 grid, regrowth 30,
# gains 4 / 20, reproduction 0.04 / 0.05 as integer thresholds floor(p * 2^32).
T_SHEEP = 171798691
T_WOLF = 214748364


def pred_params(W=64, H=64, R=30, gain_s=4, gain_w=20, T_s=T_SHEEP, T_w=T_WOLF, seed=0,
                cap_s=4096, cap_w=1024, n_s0=400, n_w0=100, multi_prey=0) -> PredParams:
    return PredParams(W, H, R, gain_s, gain_w, T_s, T_w, seed, cap_s, cap_w, n_s0, n_w0,
                      multi_prey)


@dataclass
class PredState:
    """Host copy of a predation model: grass countdown and per-species SoA."""
    grass: np.ndarray
    sheep: dict = field(default_factory=dict)   # x, y, e, alive -> int32[cap_s]
    wolves: dict = field(default_factory=dict)  # x, y, e, alive -> int32[cap_w]
    step: int = 0

    def copy(self) -> "PredState":
        return PredState(self.grass.copy(), {k: v.copy() for k, v in self.sheep.items()},
                         {k: v.copy() for k, v in self.wolves.items()}, self.step)

    def _c(self):
        def sp(d):
            return _Species(*(_ptr(d[k], C.c_int32) for k in ("x", "y", "e", "alive")))
        return _PredState(_ptr(self.grass, C.c_int32), sp(self.sheep), sp(self.wolves),
                          self.step)


def _empty_state(P: PredParams) -> PredState:
    G = P.W * P.H
    z = lambda n: np.zeros(n, dtype=np.int32)
    return PredState(z(G), {k: z(P.cap_s) for k in ("x", "y", "e", "alive")},
                     {k: z(P.cap_w) for k in ("x", "y", "e", "alive")}, 0)


def predation_init(P: PredParams) -> PredState:
    S = _empty_state(P)
    cs = S._c()
    lib().orc_predation_init(C.byref(P), C.byref(cs))
    S.step = int(cs.step)
    return S


def predation_step(P: PredParams, S: PredState) -> dict:
    """Advance S in place by one step; returns that step's statistics."""
    cs = S._c()
    st = PredStats()
    lib().orc_predation_step(C.byref(P), C.byref(cs), C.byref(st))
    S.step = int(cs.step)
    return st.as_dict()


def predation_run(P: PredParams, S: PredState, n_steps: int) -> list:
    return [predation_step(P, S) for _ in range(n_steps)]


# ---------------------------------------------------------------- single phases
# (for tests that check one phase at a time; predation_step runs all five)

def _phase(name, P, S, n_out):
    outs = [C.c_int64() for _ in range(n_out)]
    cs = S._c()
    fn = getattr(lib(), name)
    fn(C.byref(P), C.byref(cs), *[C.byref(o) for o in outs])
    return tuple(o.value for o in outs)


def pred_move(P, S):
    _phase("orc_pred_move", P, S, 0)


def pred_eat(P, S):
    """Returns (grass_eaten, sheep_eaten)."""
    return _phase("orc_pred_eat", P, S, 2)


def pred_breed(P, S):
    """Returns (births_s, births_w)."""
    return _phase("orc_pred_breed", P, S, 2)


def pred_die(P, S):
    """Returns (starved_s, starved_w)."""
    return _phase("orc_pred_die", P, S, 2)


def pred_regrow(P, S):
    _phase("orc_pred_regrow", P, S, 0)


# ---------------------------------------------------------------- sort / select
def sort_agents(attrs, key, descending=False, alive=None):
    """Returns (sorted attrs [A, n], sorted alive or None, perm int32[n])."""
    out = np.array(attrs, dtype=np.int32, order="C", copy=True)
    key = np.ascontiguousarray(key, dtype=np.int32)
    n = key.size
    assert out.shape[1] == n
    al = None if alive is None else np.array(alive, dtype=np.int32, copy=True)
    perm = np.empty(max(1, n), dtype=np.int32)
    lib().orc_sort_agents(n, out.shape[0], _ptr_array(out),
                          _ptr(al, C.c_int32) if al is not None else None,
                          _ptr(key, C.c_int32), int(bool(descending)), _ptr(perm, C.c_int32))
    return out, al, perm[:n].copy()


def select_agents(cond):
    """Returns (order int32[n]: satisfying indices first, both groups in index
    order; count)."""
    cond = np.ascontiguousarray(cond, dtype=np.uint8)
    order = np.empty(max(1, cond.size), dtype=np.int32)
    p = lib().orc_select_agents(_ptr(cond, C.c_uint8), cond.size, _ptr(order, C.c_int32))
    return order[:cond.size].copy(), int(p)


# ---------------------------------------------------------------- traffic
TRAFFIC_STATS = tuple(k for k, _ in TrafficStats._fields_)


def traffic_params(length=100, T_green=2 ** 31, T_spawn=2 ** 31, seed=0) -> TrafficParams:
    return TrafficParams(length, T_green, T_spawn, seed)


@dataclass
class TrafficState:
    """Host copy of one road: car slots (lane, pos, alive) and the step counter."""
    lane: np.ndarray
    pos: np.ndarray
    alive: np.ndarray
    step: int = 0

    def copy(self) -> "TrafficState":
        return TrafficState(self.lane.copy(), self.pos.copy(), self.alive.copy(), self.step)

    def _c(self):
        return _TrafficState(_ptr(self.lane, C.c_int32), _ptr(self.pos, C.c_int32),
                             _ptr(self.alive, C.c_int32), self.step)


def traffic_init(P: TrafficParams) -> TrafficState:
    n = 3 * P.length
    S = TrafficState(*(np.zeros(n, dtype=np.int32) for _ in range(3)))
    cs = S._c()
    lib().orc_traffic_init(C.byref(P), C.byref(cs))
    S.step = int(cs.step)
    return S


def traffic_step(P: TrafficParams, S: TrafficState) -> dict:
    cs = S._c()
    st = TrafficStats()
    lib().orc_traffic_step(C.byref(P), C.byref(cs), C.byref(st))
    S.step = int(cs.step)
    return st.as_dict()


def traffic_run(P: TrafficParams, S: TrafficState, n_steps: int) -> list:
    return [traffic_step(P, S) for _ in range(n_steps)]


# ---------------------------------------------------------------- limit order books
LOB_STATS = tuple(k for k, _ in LobStats._fields_)
LOB_FIELDS = ("side", "price", "qty", "time", "alive")


def lob_params(cap=1000, traders=10, T_order=2 ** 31, spread=20, max_qty=10, expiry=20,
               price0=10000, seed=0) -> LobParams:
    return LobParams(cap, traders, T_order, spread, max_qty, expiry, price0, seed)


@dataclass
class LobState:
    """Host copy of one book: order slots and the last price."""
    orders: dict
    last_price: int
    step: int = 0

    def copy(self) -> "LobState":
        return LobState({k: v.copy() for k, v in self.orders.items()}, self.last_price, self.step)

    def _c(self):
        return _LobState(*(_ptr(self.orders[k], C.c_int32) for k in LOB_FIELDS),
                         self.last_price, self.step)


def lob_init(P: LobParams) -> LobState:
    S = LobState({k: np.zeros(P.cap, dtype=np.int32) for k in LOB_FIELDS}, 0)
    cs = S._c()
    lib().orc_lob_init(C.byref(P), C.byref(cs))
    S.last_price, S.step = int(cs.last_price), int(cs.step)
    return S


def lob_step(P: LobParams, S: LobState) -> dict:
    cs = S._c()
    st = LobStats()
    lib().orc_lob_step(C.byref(P), C.byref(cs), C.byref(st))
    S.last_price, S.step = int(cs.last_price), int(cs.step)
    return st.as_dict()


def lob_run(P: LobParams, S: LobState, n_steps: int) -> list:
    return [lob_step(P, S) for _ in range(n_steps)]
