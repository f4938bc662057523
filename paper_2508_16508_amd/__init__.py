"""Python binding for libabm.so, the MI355X (gfx950) ABMax hot path.

Argument marshalling only: every step of the path runs in the HIP kernels of
``libabm.so``; PyTorch supplies device memory and the current stream.  The
names follow the C ABI in ``include/abm.h``.  Importing this package does not
need a GPU; calling into it does, and a missing library is an error (there is
no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libabm.so")

ABM_MAX_ATTRS = 16
ABM_OK, ABM_E_INVALID, ABM_E_WORKSPACE, ABM_E_HIP, ABM_E_UNSUPPORTED = 0, -1, -2, -3, -4
ABM_OP_SELECT_UPDATE, ABM_OP_ADD_AGENTS, ABM_OP_REMOVE_AGENTS = 1, 2, 3
ABM_OP_SELECT_INDICES, ABM_OP_PREDATION = 4, 5

# Every symbol include/abm.h declares.
EXPORTED = (
    "abm_workspace_bytes", "abm_workspace_init", "abm_select_update", "abm_select_indices",
    "abm_add_agents", "abm_remove_agents", "abm_resolve_conflicts", "abm_predation_init",
    "abm_predation_step", "abm_last_error", "abm_version", "abm_batched_workspace_bytes",
    "abm_predation_batched_init", "abm_predation_run_batched", "abm_predation_batched_grass",
    "abm_select_update_batched", "abm_add_agents_batched", "abm_remove_agents_batched",
    "abm_resolve_conflicts_batched", "abm_traffic_init", "abm_traffic_step",
    "abm_sort_workspace_bytes", "abm_sort_agents", "abm_select_agents", "abm_lob_init",
    "abm_lob_step", "abm_predation_batched_graph", "abm_graph_replay", "abm_graph_destroy",
    "abm_batched_lds_cells",
    "abm_select_update_noalloc",
)


class AbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"abm status {code}: {msg}")
        self.code = code


class Soa(C.Structure):
    _fields_ = [("n_attrs", C.c_int32), ("capacity", C.c_int64),
                ("attr", C.c_void_p * ABM_MAX_ATTRS), ("alive", C.c_void_p)]


class Records(C.Structure):
    _fields_ = [("n_attrs", C.c_int32), ("count", C.c_int64),
                ("attr", C.c_void_p * ABM_MAX_ATTRS)]


class PredationParams(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("R", C.c_int32),
                ("gain_s", C.c_int32), ("gain_w", C.c_int32),
                ("T_s", C.c_uint32), ("T_w", C.c_uint32), ("seed", C.c_uint32),
                ("cap_s", C.c_int64), ("cap_w", C.c_int64),
                ("n_s0", C.c_int64), ("n_w0", C.c_int64), ("multi_prey", C.c_int32)]


class LobParams(C.Structure):
    _fields_ = [("cap", C.c_int32), ("traders", C.c_int32), ("T_order", C.c_uint32),
                ("spread", C.c_int32), ("max_qty", C.c_int32), ("expiry", C.c_int32),
                ("price0", C.c_int32), ("seed", C.c_uint32)]


class LobStatePtrs(C.Structure):
    _fields_ = [("n_books", C.c_int32), ("side", C.c_void_p), ("price", C.c_void_p),
                ("qty", C.c_void_p), ("time", C.c_void_p), ("alive", C.c_void_p),
                ("last_price", C.c_void_p), ("stats", C.c_void_p), ("step", C.c_uint32)]


class TrafficParams(C.Structure):
    _fields_ = [("length", C.c_int32), ("T_green", C.c_uint32), ("T_spawn", C.c_uint32),
                ("seed", C.c_uint32)]


class TrafficStatePtrs(C.Structure):
    _fields_ = [("n_roads", C.c_int32), ("lane", C.c_void_p), ("pos", C.c_void_p),
                ("alive", C.c_void_p), ("stats", C.c_void_p), ("step", C.c_uint32)]


class SpeciesPtrs(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("e", C.c_void_p), ("alive", C.c_void_p)]


class PredationStatePtrs(C.Structure):
    _fields_ = [("grass", C.c_void_p), ("sheep", SpeciesPtrs), ("wolves", SpeciesPtrs),
                ("claims", C.c_void_p), ("stats", C.c_void_p), ("step", C.c_uint32)]


class Batch(C.Structure):
    _fields_ = [("n_models", C.c_int32), ("max_cap", C.c_int64), ("models", C.c_void_p),
                ("ready", C.c_void_p), ("claims", C.c_void_p), ("sheep", SpeciesPtrs),
                ("wolves", SpeciesPtrs), ("link_s", C.c_void_p), ("link_w", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("block_threads", C.c_int32), ("workgroups", C.c_int32), ("items", C.c_int32),
                ("team_size", C.c_int32), ("team_models", C.c_int32),
                ("team_workgroups", C.c_int32), ("global_claims", C.c_int32)]


_lib = None


def lib():
    """The loaded libabm.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950) first")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
        L.abm_workspace_bytes.argtypes = [C.c_int, i64]
        L.abm_workspace_bytes.restype = sz
        L.abm_workspace_init.argtypes = [vp, sz, vp]
        L.abm_select_update.argtypes = [C.POINTER(Soa), vp, C.POINTER(Records), vp, vp, vp, vp,
                                        sz, vp]
        L.abm_select_indices.argtypes = [vp, i64, vp, vp, vp, sz, vp]
        L.abm_select_update_noalloc.argtypes = [C.POINTER(Soa), vp, C.POINTER(Records), vp, vp,
                                                vp, vp]
        L.abm_add_agents.argtypes = [C.POINTER(Soa), C.POINTER(Records), vp, vp, vp, sz, vp]
        L.abm_remove_agents.argtypes = [C.POINTER(Soa), vp, vp, vp, sz, vp]
        L.abm_resolve_conflicts.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp]
        L.abm_predation_init.argtypes = [C.POINTER(PredationParams),
                                         C.POINTER(PredationStatePtrs), vp]
        L.abm_predation_step.argtypes = [C.POINTER(PredationParams),
                                         C.POINTER(PredationStatePtrs), i32, vp, sz, vp]
        L.abm_batched_workspace_bytes.argtypes = [i64, i32]
        L.abm_batched_workspace_bytes.restype = sz
        L.abm_predation_batched_init.argtypes = [C.POINTER(Batch), vp]
        L.abm_batched_lds_cells.argtypes = [i32, i32]
        L.abm_batched_lds_cells.restype = i64
        L.abm_predation_run_batched.argtypes = [C.POINTER(Batch), vp, i32, C.POINTER(Tuning), vp,
                                                sz, vp]
        L.abm_predation_batched_grass.argtypes = [C.POINTER(Batch), vp, vp]
        L.abm_predation_batched_graph.argtypes = [C.POINTER(Batch), vp, i32, i32,
                                                  C.POINTER(Tuning), vp, sz, C.POINTER(vp)]
        L.abm_graph_replay.argtypes = [vp, vp]
        L.abm_graph_destroy.argtypes = [vp]
        L.abm_select_update_batched.argtypes = [i32, C.POINTER(Soa), vp, vp, C.POINTER(Records), vp,
                                                vp, vp, vp, sz, vp]
        L.abm_add_agents_batched.argtypes = [i32, C.POINTER(Soa), vp, C.POINTER(Records), vp, vp,
                                             vp, vp, sz, vp]
        L.abm_remove_agents_batched.argtypes = [i32, C.POINTER(Soa), vp, vp, vp, vp, sz, vp]
        L.abm_resolve_conflicts_batched.argtypes = [i32, vp, i64, vp, vp, vp, vp, i64, vp, vp, vp,
                                                    vp]
        L.abm_sort_workspace_bytes.argtypes = [i64, i32]
        L.abm_sort_workspace_bytes.restype = sz
        L.abm_sort_agents.argtypes = [C.POINTER(Soa), vp, i32, vp, vp, sz, vp]
        L.abm_select_agents.argtypes = [vp, i64, vp, vp, vp, sz, vp]
        L.abm_lob_init.argtypes = [C.POINTER(LobParams), C.POINTER(LobStatePtrs), vp]
        L.abm_lob_step.argtypes = [C.POINTER(LobParams), C.POINTER(LobStatePtrs), i32, vp]
        L.abm_traffic_init.argtypes = [C.POINTER(TrafficParams), C.POINTER(TrafficStatePtrs), vp]
        L.abm_traffic_step.argtypes = [C.POINTER(TrafficParams), C.POINTER(TrafficStatePtrs), i32,
                                       vp]
        L.abm_last_error.restype = C.c_char_p
        L.abm_version.restype = C.c_char_p
        for name in EXPORTED:
            if name not in ("abm_workspace_bytes", "abm_last_error", "abm_version",
                            "abm_batched_workspace_bytes", "abm_sort_workspace_bytes"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != ABM_OK:
        raise AbmError(rc, lib().abm_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require(t, dtype, name):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _rows(t: torch.Tensor, name: str):
    """Row pointers of a 2-D int32 tensor [n_attrs, length] (or a list of 1-D tensors)."""
    if isinstance(t, (list, tuple)):
        for r in t:
            _require(r, torch.int32, name)
        return [r.data_ptr() for r in t], (t[0].numel() if len(t) else 0)
    _require(t, torch.int32, name)
    if t.dim() != 2:
        raise ValueError(f"{name} must be [n_attrs, length]")
    return [t[a].data_ptr() for a in range(t.shape[0])], t.shape[1]


def make_soa(attrs, alive=None) -> Soa:
    ptrs, n = _rows(attrs, "attrs")
    s = Soa()
    s.n_attrs = len(ptrs)
    s.capacity = n if ptrs else (alive.numel() if alive is not None else 0)
    for a, p in enumerate(ptrs):
        s.attr[a] = p
    _require(alive, torch.int32, "alive")
    s.alive = alive.data_ptr() if alive is not None else None
    return s


def make_records(recs) -> Records:
    ptrs, m = _rows(recs, "records")
    r = Records()
    r.n_attrs = len(ptrs)
    r.count = m
    for a, p in enumerate(ptrs):
        r.attr[a] = p
    return r


def workspace_bytes(op: int, capacity: int) -> int:
    return int(lib().abm_workspace_bytes(op, capacity))


def workspace(capacity: int, op: int = ABM_OP_PREDATION, device=None, stream=None) -> torch.Tensor:
    """Allocate and initialise a workspace big enough for `capacity` slots."""
    nbytes = workspace_bytes(op, capacity)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    ws = ws[off: off + nbytes]
    _check(lib().abm_workspace_init(_p(ws), nbytes, _stream(stream)))
    return ws


def workspace_error(ws: torch.Tensor) -> int:
    """The workspace error word: non-zero if a bounded wait inside a kernel ever
    gave up (the single-pass scan's ordering assumption failed).  Synchronises."""
    return int(ws[248:256].view(torch.int64).item())


def _counts(device, *given):
    return [g if g is not None else torch.zeros(1, dtype=torch.int64, device=device) for g in given]


def select_update(attrs, sel_mask, recs, upd_mask=None, ws=None, applied=None, dropped=None,
                  stream=None):
    """Distinct updates to the selected slots (Sec. 4).  Returns (applied, dropped)
    as 1-element int64 device tensors; attrs is updated in place."""
    dst = make_soa(attrs)
    upd = make_records(recs)
    _require(sel_mask, torch.uint8, "sel_mask")
    _require(upd_mask, torch.uint8, "upd_mask")
    dev = sel_mask.device
    if ws is None:
        ws = workspace(max(dst.capacity, upd.count), ABM_OP_SELECT_UPDATE, dev, stream)
    applied, dropped = _counts(dev, applied, dropped)
    _check(lib().abm_select_update(C.byref(dst), _p(sel_mask), C.byref(upd), _p(upd_mask),
                                   _p(applied), _p(dropped), _p(ws), ws.numel(), _stream(stream)))
    return applied, dropped


def select_update_noalloc(attrs, sel_mask, recs, applied=None, dropped=None, error=None,
                          stream=None):
    """select_update with dense records and no workspace (the library's
    static scan state; at most 2^28 slots; calls on one device must not
    overlap).  Returns (applied, dropped, error) device int64 tensors."""
    dst = make_soa(attrs)
    upd = make_records(recs)
    _require(sel_mask, torch.uint8, "sel_mask")
    applied, dropped, error = _counts(sel_mask.device, applied, dropped, error)
    _check(lib().abm_select_update_noalloc(C.byref(dst), _p(sel_mask), C.byref(upd), _p(applied),
                                           _p(dropped), _p(error), _stream(stream)))
    return applied, dropped, error


def select_indices(mask, out_idx=None, ws=None, count=None, stream=None):
    """Ascending indices of the selected entries (Sec. 2 select_agents).
    Returns (out_idx int32[n], count int64[1]); entries [0, count) are valid."""
    _require(mask, torch.uint8, "mask")
    n = mask.numel()
    dev = mask.device
    if out_idx is None:
        out_idx = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(n, ABM_OP_SELECT_INDICES, dev, stream)
    (count,) = _counts(dev, count)
    _check(lib().abm_select_indices(_p(mask), n, _p(out_idx), _p(count), _p(ws), ws.numel(),
                                    _stream(stream)))
    return out_idx, count


def sort_workspace(n: int, device="cuda", n_cols: int = 0) -> torch.Tensor:
    """A 256-byte-aligned workspace for sort_agents over n agents permuting
    n_cols columns (attributes plus alive), or for select_agents (n_cols 0)."""
    nbytes = int(lib().abm_sort_workspace_bytes(n, n_cols))
    if nbytes == 0:
        raise ValueError(f"no sort workspace for n = {n}, n_cols = {n_cols}")
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off: off + nbytes]


def sort_agents(attrs, key, descending=False, alive=None, perm=None, ws=None, stream=None):
    """Reorder the collection in place by a runtime int32 key (Sec. 2
    sort_agents; stable, ascending or descending).  Returns perm int32[n]: the
    old index of the agent now at each position."""
    _require(key, torch.int32, "key")
    dst = make_soa(attrs, alive)
    dst.capacity = key.numel()
    dev = key.device
    if perm is None:
        perm = torch.empty(max(1, key.numel()), dtype=torch.int32, device=dev)
    if ws is None:
        ws = sort_workspace(key.numel(), dev, dst.n_attrs + (alive is not None))
    _check(lib().abm_sort_agents(C.byref(dst), _p(key), int(bool(descending)), _p(perm), _p(ws),
                                 ws.numel(), _stream(stream)))
    return perm


def select_agents(cond, order=None, ws=None, count=None, stream=None):
    """Sec. 2 select_agents: (order int32[n] -- the indices satisfying cond in
    increasing order, then the others -- and count int64[1])."""
    _require(cond, torch.uint8, "cond")
    n = cond.numel()
    dev = cond.device
    if order is None:
        order = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    if ws is None:
        ws = sort_workspace(n, dev)
    (count,) = _counts(dev, count)
    _check(lib().abm_select_agents(_p(cond), n, _p(order), _p(count), _p(ws), ws.numel(),
                                   _stream(stream)))
    return order, count


def add_agents(attrs, alive, recs, ws=None, added=None, dropped=None, stream=None):
    """Newborn j into the j-th lowest free slot.  Returns (added, dropped)."""
    dst = make_soa(attrs, alive)
    nb = make_records(recs)
    dev = alive.device
    if ws is None:
        ws = workspace(dst.capacity, ABM_OP_ADD_AGENTS, dev, stream)
    added, dropped = _counts(dev, added, dropped)
    _check(lib().abm_add_agents(C.byref(dst), C.byref(nb), _p(added), _p(dropped), _p(ws),
                                ws.numel(), _stream(stream)))
    return added, dropped


def remove_agents(alive, kill_mask, ws=None, removed=None, stream=None):
    """alive[i] = 0 wherever kill_mask[i] (Sec. 2 set_agents_mask).  Returns removed."""
    _require(alive, torch.int32, "alive")
    _require(kill_mask, torch.uint8, "kill_mask")
    s = Soa()
    s.n_attrs = 0
    s.capacity = alive.numel()
    s.alive = alive.data_ptr()
    dev = alive.device
    if ws is None:
        ws = workspace(alive.numel(), ABM_OP_REMOVE_AGENTS, dev, stream)
    (removed,) = _counts(dev, removed)
    _check(lib().abm_remove_agents(C.byref(s), _p(kill_mask), _p(removed), _p(ws), ws.numel(),
                                   _stream(stream)))
    return removed


def resolve_conflicts(target, prio, n_targets, active=None, best=None, winner=None, won=None,
                      stream=None):
    """Lowest (prio, claim) wins each target.  Returns (best, winner, won)."""
    _require(target, torch.int32, "target")
    _require(prio, torch.int32 if prio.dtype == torch.int32 else torch.uint32, "prio")
    _require(active, torch.uint8, "active")
    n = target.numel()
    dev = target.device
    if best is None:
        best = torch.empty(max(1, n_targets), dtype=torch.uint64, device=dev)
    if winner is None:
        winner = torch.empty(max(1, n_targets), dtype=torch.int32, device=dev)
    if won is None:
        won = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    _check(lib().abm_resolve_conflicts(n, _p(target), _p(prio), _p(active), n_targets, _p(best),
                                       _p(winner), _p(won), _stream(stream)))
    return best, winner, won


# ---------------------------------------------------------------- batched primitives

def _offsets(off, name):
    _require(off, torch.int64, name)
    return off.numel() - 1


def select_update_batched(attrs, slot_off, sel_mask, recs, rec_off, ws=None, applied=None,
                          dropped=None, stream=None):
    """select_update on every segment of packed collections (device offsets).
    Returns per-segment (applied, dropped) int64 device tensors."""
    n_seg = _offsets(slot_off, "slot_off")
    _offsets(rec_off, "rec_off")
    dst, upd = make_soa(attrs), make_records(recs)
    _require(sel_mask, torch.uint8, "sel_mask")
    dev = slot_off.device
    if ws is None:
        ws = workspace(dst.capacity, ABM_OP_SELECT_UPDATE, dev, stream)
    applied = applied if applied is not None else torch.zeros(max(1, n_seg), dtype=torch.int64,
                                                               device=dev)
    dropped = dropped if dropped is not None else torch.zeros(max(1, n_seg), dtype=torch.int64,
                                                               device=dev)
    _check(lib().abm_select_update_batched(n_seg, C.byref(dst), _p(slot_off), _p(sel_mask),
                                           C.byref(upd), _p(rec_off), _p(applied), _p(dropped),
                                           _p(ws), ws.numel(), _stream(stream)))
    return applied, dropped


def add_agents_batched(attrs, alive, slot_off, recs, rec_off, ws=None, stream=None):
    n_seg = _offsets(slot_off, "slot_off")
    _offsets(rec_off, "rec_off")
    dst, nb = make_soa(attrs, alive), make_records(recs)
    dev = slot_off.device
    if ws is None:
        ws = workspace(dst.capacity, ABM_OP_ADD_AGENTS, dev, stream)
    added = torch.zeros(max(1, n_seg), dtype=torch.int64, device=dev)
    dropped = torch.zeros(max(1, n_seg), dtype=torch.int64, device=dev)
    _check(lib().abm_add_agents_batched(n_seg, C.byref(dst), _p(slot_off), C.byref(nb),
                                        _p(rec_off), _p(added), _p(dropped), _p(ws), ws.numel(),
                                        _stream(stream)))
    return added, dropped


def remove_agents_batched(alive, slot_off, kill_mask, ws=None, stream=None):
    n_seg = _offsets(slot_off, "slot_off")
    _require(alive, torch.int32, "alive")
    _require(kill_mask, torch.uint8, "kill_mask")
    s = Soa()
    s.n_attrs = 0
    s.capacity = alive.numel()
    s.alive = alive.data_ptr()
    dev = slot_off.device
    if ws is None:
        ws = workspace(alive.numel(), ABM_OP_REMOVE_AGENTS, dev, stream)
    removed = torch.zeros(max(1, n_seg), dtype=torch.int64, device=dev)
    _check(lib().abm_remove_agents_batched(n_seg, C.byref(s), _p(slot_off), _p(kill_mask),
                                           _p(removed), _p(ws), ws.numel(), _stream(stream)))
    return removed


def resolve_conflicts_batched(claim_off, target, prio, target_off, active=None, stream=None):
    """Returns packed (best, winner, won); winner holds segment-local claim indices."""
    n_seg = _offsets(claim_off, "claim_off")
    _offsets(target_off, "target_off")
    n = target.numel()
    nt = int(target_off[-1].item())
    dev = target.device
    best = torch.empty(max(1, nt), dtype=torch.uint64, device=dev)
    winner = torch.empty(max(1, nt), dtype=torch.int32, device=dev)
    won = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    _check(lib().abm_resolve_conflicts_batched(n_seg, _p(claim_off), n, _p(target), _p(prio),
                                               _p(active), _p(target_off), nt, _p(best),
                                               _p(winner), _p(won), _stream(stream)))
    return best, winner, won


# ---------------------------------------------------------------- predation

@dataclass
class PredationModel:
    """Device-resident predation model (Sec. 5.1): grass countdown, per-species
    SoA (x, y, energy, alive) and the per-cell claim tables."""
    params: PredationParams
    grass: torch.Tensor
    sheep: dict
    wolves: dict
    claims: torch.Tensor
    ws: torch.Tensor
    step: int = 0

    @staticmethod
    def create(params: PredationParams, device="cuda", stream=None) -> "PredationModel":
        G = params.W * params.H
        z = lambda n: torch.empty(n, dtype=torch.int32, device=device)
        sheep = {k: z(params.cap_s) for k in ("x", "y", "e", "alive")}
        wolves = {k: z(params.cap_w) for k in ("x", "y", "e", "alive")}
        claims = torch.empty(3 * G, dtype=torch.uint64, device=device)
        ws = workspace(max(params.cap_s, params.cap_w), ABM_OP_PREDATION, device, stream)
        return PredationModel(params, z(G), sheep, wolves, claims, ws)

    def _ptrs(self, stats=None) -> PredationStatePtrs:
        sp = lambda d: SpeciesPtrs(*(d[k].data_ptr() for k in ("x", "y", "e", "alive")))
        return PredationStatePtrs(self.grass.data_ptr(), sp(self.sheep), sp(self.wolves),
                                  self.claims.data_ptr(),
                                  stats.data_ptr() if stats is not None else None, self.step)

    def init(self, stream=None):
        st = self._ptrs()
        _check(lib().abm_predation_init(C.byref(self.params), C.byref(st), _stream(stream)))
        self.step = int(st.step)

    def run(self, n_steps: int, stats: torch.Tensor | None = None, stream=None):
        """Advance n_steps; stats (int64 [n_steps, 8]) receives per-step counts."""
        if stats is not None:
            _require(stats, torch.int64, "stats")
            assert stats.numel() >= 8 * n_steps
        st = self._ptrs(stats)
        _check(lib().abm_predation_step(C.byref(self.params), C.byref(st), n_steps,
                                        _p(self.ws), self.ws.numel(), _stream(stream)))
        self.step = int(st.step)


def predation_params(W=64, H=64, R=30, gain_s=4, gain_w=20, T_s=171798691, T_w=214748364,
                     seed=0, cap_s=4096, cap_w=1024, n_s0=400, n_w0=100,
                     multi_prey=0) -> PredationParams:
    """Defaults: the small 64x64 workload (regrowth 30, gains 4 / 20,
    reproduction 0.04 / 0.05 as floor(p * 2^32)).  multi_prey = 1: wolves and
    sheep of a cell are matched by rank."""
    return PredationParams(W, H, R, gain_s, gain_w, T_s, T_w, seed, cap_s, cap_w, n_s0, n_w0,
                           multi_prey)


def predation_init(params, model: PredationModel | None = None, device="cuda", stream=None):
    m = model or PredationModel.create(params, device, stream)
    m.init(stream)
    return m


def predation_step(model: PredationModel, n_steps: int = 1, stats=None, stream=None):
    model.run(n_steps, stats, stream)
    return model


STAT_NAMES = ("live_s", "live_w", "grass_eaten", "sheep_eaten", "births_s", "births_w",
              "starved_s", "starved_w")


# ---------------------------------------------------------------- batched predation

class ModelDesc(C.Structure):
    """Mirror of abm_model_desc."""
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("R", C.c_int32),
                ("gain_s", C.c_int32), ("gain_w", C.c_int32),
                ("T_s", C.c_uint32), ("T_w", C.c_uint32), ("seed", C.c_uint32),
                ("multi_prey", C.c_int32), ("cap_s", C.c_int64), ("cap_w", C.c_int64),
                ("n_s0", C.c_int64), ("n_w0", C.c_int64),
                ("cell_off", C.c_int64), ("sheep_off", C.c_int64), ("wolf_off", C.c_int64),
                ("step", C.c_int32), ("steps_target", C.c_int32),
                ("updates", C.c_int64), ("live_s", C.c_int64), ("live_w", C.c_int64)]


class BatchedPredation:
    """Many predation models of uneven sizes, packed for one persistent launch.

    models: list of PredationParams (one per model); steps_target: per model
    (int or list).  Slot and cell ranges are packed in model order; the launch
    order is largest model first.  Models of at least team_min_size cells plus
    slots are each advanced by a team of team_size workgroups (team_size 1: no
    teams).  With lds=True models of one workgroup whose claim table fits the
    workgroup's LDS (lds_cells()) keep it there."""

    def __init__(self, models, steps_target, device="cuda", block_threads=512, items=4,
                 team_size=1, team_min_size=1 << 18, lds=True):
        self.params = list(models)
        n = len(self.params)
        tgt = [steps_target] * n if isinstance(steps_target, int) else list(steps_target)
        self.n_models = n
        descs = (ModelDesc * max(1, n))()
        g_off = s_off = w_off = 0
        for m, p in enumerate(self.params):
            d = descs[m]
            for f in ("W", "H", "R", "gain_s", "gain_w", "T_s", "T_w", "seed", "multi_prey",
                      "cap_s", "cap_w", "n_s0", "n_w0"):
                setattr(d, f, getattr(p, f))
            d.cell_off, d.sheep_off, d.wolf_off = g_off, s_off, w_off
            d.step, d.steps_target = 0, int(tgt[m])
            g_off += p.W * p.H
            s_off += p.cap_s
            w_off += p.cap_w
        self.cells, self.slots_s, self.slots_w = g_off, s_off, w_off
        self.max_cap = max([max(p.cap_s, p.cap_w) for p in self.params] or [1])
        z = lambda k: torch.zeros(max(1, k), dtype=torch.int32, device=device)
        self.ready = z(g_off)
        self.claims = torch.empty(3 * max(1, g_off), dtype=torch.uint64, device=device)
        self.sheep = {f: z(s_off) for f in ("x", "y", "e", "alive")}
        self.wolves = {f: z(w_off) for f in ("x", "y", "e", "alive")}
        # per-cell list links, needed only by multi-prey models
        multi = any(p.multi_prey for p in self.params)
        self.links = (z(s_off), z(w_off)) if multi else None
        raw = bytes(descs)
        self.desc = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
        size = [p.W * p.H + p.cap_s + p.cap_w for p in self.params]
        order = sorted(range(n), key=lambda m: -size[m])
        self.order = torch.tensor(order or [0], dtype=torch.int32, device=device)
        self.size = size
        self.sorted_size = [size[m] for m in order]
        self.lds = lds
        self.block_threads = block_threads
        self.items = items
        self.team_size = team_size
        self.team_min_size = team_min_size
        props = torch.cuda.get_device_properties(self.ready.device)
        self.workgroups = props.multi_processor_count * max(1, 2048 // block_threads)
        nbytes = int(lib().abm_batched_workspace_bytes(self.max_cap, self.workgroups))
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off: off + nbytes]
        # zeroed once: the error word at its end of the header is sticky
        _check(lib().abm_workspace_init(_p(self.ws), nbytes, _stream()))

    def _batch(self) -> Batch:
        sp = lambda d: SpeciesPtrs(*(d[k].data_ptr() for k in ("x", "y", "e", "alive")))
        ls, lw = (t.data_ptr() for t in self.links) if self.links else (None, None)
        return Batch(self.n_models, self.max_cap, self.desc.data_ptr(), self.ready.data_ptr(),
                     self.claims.data_ptr(), sp(self.sheep), sp(self.wolves), ls, lw)

    def init(self, stream=None):
        b = self._batch()
        _check(lib().abm_predation_batched_init(C.byref(b), _stream(stream)))

    def lds_cells(self, block_threads=None, items=None) -> int:
        """Largest W * H whose claims stay in LDS at this launch shape (0: none)."""
        if not self.lds:
            return 0
        return int(lib().abm_batched_lds_cells(block_threads or self.block_threads,
                                               items or self.items))

    def lds_models(self, block_threads=None, items=None) -> int:
        """Models that keep their claims in LDS at this launch shape (no teams)."""
        lim = self.lds_cells(block_threads, items)
        return sum(1 for p in self.params if p.W * p.H <= lim)

    def team_models(self, team_min_size=None) -> int:
        """Number of leading models of the launch order big enough for a team."""
        lim = self.team_min_size if team_min_size is None else team_min_size
        return sum(1 for v in self.sorted_size if v >= lim)

    def run(self, max_steps: int, stream=None, block_threads=None, workgroups=None, items=None,
            team_size=None, team_min_size=None, team_workgroups=0):
        b = self._batch()
        t = self._tuning(block_threads, workgroups, items, team_size, team_min_size,
                         team_workgroups)
        _check(lib().abm_predation_run_batched(C.byref(b), _p(self.order), max_steps, C.byref(t),
                                               _p(self.ws), self.ws.numel(), _stream(stream)))

    def _tuning(self, block_threads=None, workgroups=None, items=None, team_size=None,
                team_min_size=None, team_workgroups=0) -> Tuning:
        k = self.team_size if team_size is None else team_size
        nt = self.team_models(team_min_size) if k > 1 else 0
        return Tuning(block_threads or self.block_threads, workgroups or self.workgroups,
                      items or self.items, k, nt, team_workgroups, 0 if self.lds else 1)

    def capture(self, chunk_steps: int, n_chunks: int, **tuning) -> "RolloutGraph":
        """A rollout of n_chunks launches of up to chunk_steps steps each,
        captured by the library as one graph (nothing runs until replay)."""
        b = self._batch()
        t = self._tuning(**tuning)
        h = C.c_void_p()
        _check(lib().abm_predation_batched_graph(C.byref(b), _p(self.order), chunk_steps,
                                                 n_chunks, C.byref(t), _p(self.ws),
                                                 self.ws.numel(), C.byref(h)))
        return RolloutGraph(h, self)

    def descriptors(self):
        """Host copy of the model descriptors (synchronises)."""
        raw = self.desc.cpu().numpy().tobytes()
        return (ModelDesc * max(1, self.n_models)).from_buffer_copy(raw)[: self.n_models]

    def grass_countdown(self, stream=None) -> torch.Tensor:
        out = torch.zeros(max(1, self.cells), dtype=torch.int32, device=self.ready.device)
        b = self._batch()
        _check(lib().abm_predation_batched_grass(C.byref(b), _p(out), _stream(stream)))
        return out

    def model_state(self, m: int, countdown: torch.Tensor | None = None):
        """(grass countdown, sheep dict, wolves dict) of model m as device views."""
        p = self.params[m]
        dm = self.descriptors()[m]
        g = countdown if countdown is not None else self.grass_countdown()
        grass = g[dm.cell_off: dm.cell_off + p.W * p.H]
        sheep = {k: v[dm.sheep_off: dm.sheep_off + p.cap_s] for k, v in self.sheep.items()}
        wolves = {k: v[dm.wolf_off: dm.wolf_off + p.cap_w] for k, v in self.wolves.items()}
        return grass, sheep, wolves


class RolloutGraph:
    """A captured batched rollout (abm_predation_batched_graph).  Holds the
    batch it was captured from, whose buffers the graph uses as they are."""

    def __init__(self, handle: C.c_void_p, batch: BatchedPredation):
        self.handle, self.batch = handle, batch

    def replay(self, stream=None):
        _check(lib().abm_graph_replay(self.handle, _stream(stream)))

    def destroy(self):
        if self.handle:
            _check(lib().abm_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.abm_graph_destroy(self.handle)
            self.handle = None


# ---------------------------------------------------------------- traffic
TRAFFIC_STAT_NAMES = ("cars", "exited", "moved", "blocked", "lost", "waiting_red", "spawned",
                      "lane_changes")


def traffic_params(length=100, T_green=2 ** 31, T_spawn=2 ** 31, seed=0) -> TrafficParams:
    """Traffic CA of Sec. 5.2: 3 lanes x `length` cells; lights and spawns
    succeed when a draw is below the threshold (2^31: probability 1/2)."""
    return TrafficParams(length, T_green, T_spawn, seed)


class TrafficRoads:
    """n_roads roads of one length, device-resident: car slots (lane, pos,
    alive) as int32 [n_roads, 3 * length]; road r draws with seed + r."""

    def __init__(self, params: TrafficParams, n_roads: int, device="cuda"):
        self.params = params
        self.n_roads = n_roads
        n = 3 * params.length
        z = lambda: torch.zeros((n_roads, n), dtype=torch.int32, device=device)
        self.lane, self.pos, self.alive = z(), z(), z()
        self.step = 0

    def _ptrs(self, stats=None) -> TrafficStatePtrs:
        return TrafficStatePtrs(self.n_roads, self.lane.data_ptr(), self.pos.data_ptr(),
                                self.alive.data_ptr(),
                                stats.data_ptr() if stats is not None else None, self.step)

    def init(self, stream=None):
        st = self._ptrs()
        _check(lib().abm_traffic_init(C.byref(self.params), C.byref(st), _stream(stream)))
        self.step = int(st.step)

    def run(self, n_steps: int, stats: torch.Tensor | None = None, stream=None):
        """Advance every road n_steps; stats (int64 [n_steps, n_roads, 8])
        receives per-step counts (TRAFFIC_STAT_NAMES)."""
        if stats is not None:
            _require(stats, torch.int64, "stats")
            assert stats.numel() >= 8 * n_steps * self.n_roads
        st = self._ptrs(stats)
        _check(lib().abm_traffic_step(C.byref(self.params), C.byref(st), n_steps,
                                      _stream(stream)))
        self.step = int(st.step)


# ---------------------------------------------------------------- limit order books
LOB_STAT_NAMES = ("buys", "sells", "placed", "dropped", "expired", "volume", "filled_orders",
                  "price")
LOB_FIELDS = ("side", "price", "qty", "time", "alive")


def lob_params(cap=1000, traders=10, T_order=2 ** 31, spread=20, max_qty=10, expiry=20,
               price0=10000, seed=0) -> LobParams:
    """Noisy traders on limit order books (Sec. 5.3); prices in ticks."""
    return LobParams(cap, traders, T_order, spread, max_qty, expiry, price0, seed)


class OrderBooks:
    """n_books books of one capacity, device-resident: order slots
    (side, price, qty, time, alive) as int32 [n_books, cap] and the last price
    per book; book b draws with seed + b."""

    def __init__(self, params: LobParams, n_books: int, device="cuda"):
        self.params = params
        self.n_books = n_books
        self.orders = {f: torch.zeros((n_books, params.cap), dtype=torch.int32, device=device)
                       for f in LOB_FIELDS}
        self.last_price = torch.zeros(n_books, dtype=torch.int32, device=device)
        self.step = 0

    def _ptrs(self, stats=None) -> LobStatePtrs:
        return LobStatePtrs(self.n_books, *(self.orders[f].data_ptr() for f in LOB_FIELDS),
                            self.last_price.data_ptr(),
                            stats.data_ptr() if stats is not None else None, self.step)

    def init(self, stream=None):
        st = self._ptrs()
        _check(lib().abm_lob_init(C.byref(self.params), C.byref(st), _stream(stream)))
        self.step = int(st.step)

    def run(self, n_steps: int, stats: torch.Tensor | None = None, stream=None):
        """Advance every book n_steps; stats (int64 [n_steps, n_books, 8])
        receives per-step counts (LOB_STAT_NAMES)."""
        if stats is not None:
            _require(stats, torch.int64, "stats")
            assert stats.numel() >= 8 * n_steps * self.n_books
        st = self._ptrs(stats)
        _check(lib().abm_lob_step(C.byref(self.params), C.byref(st), n_steps, _stream(stream)))
        self.step = int(st.step)
