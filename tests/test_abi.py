"""The C-ABI boundary, checked without a GPU: the library loads, exports exactly
the entry points include/abm.h declares, and rejects bad arguments on the host
before anything is launched."""
import ctypes as C
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "abm.h")


def _declared():
    text = open(HEADER).read()
    return set(re.findall(r"ABM_API\s+[\w\s\*]*?\b(abm_\w+)\s*\(", text))


def test_header_declares_binding_names(abm):
    assert _declared() == set(abm.EXPORTED)


def test_library_exports_every_declared_symbol(abm):
    out = subprocess.run(["nm", "-D", "--defined-only", abm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(abm_\w+)$", out, flags=re.M))
    assert exported == _declared()
    for name in _declared():
        assert getattr(abm.lib(), name) is not None


def test_library_is_gfx950_only(abm):
    """The offload bundle of the library (built here) targets gfx950 only."""
    blob = open(abm.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-+(gfx\w+)", blob))
    assert targets == {b"gfx950"}


def test_workspace_bytes(abm):
    small = abm.workspace_bytes(abm.ABM_OP_SELECT_UPDATE, 1)
    big = abm.workspace_bytes(abm.ABM_OP_SELECT_UPDATE, 1 << 24)
    assert 256 < small < big
    assert abm.workspace_bytes(abm.ABM_OP_PREDATION, 1 << 24) == big
    assert abm.workspace_bytes(999, 10) == 0
    assert abm.lib().abm_version().decode().startswith("abm")


def test_sort_workspace_bytes(abm):
    """Permutation + max(three 4n buffers, n records of n_cols int32 rounded up
    to a power of two) + tile counts, each part rounded up to 256 bytes."""
    f = abm.lib().abm_sort_workspace_bytes
    r = lambda b: (b + 255) // 256 * 256
    n = 1 << 24
    tiles = r(4 * 256 * (n // 4096)) + 2 * r(1024)
    assert f(n, 0) == r(4 * n) + 3 * r(4 * n) + tiles
    assert f(n, 2) == f(n, 0)                   # 8-byte records fit the three buffers
    assert f(n, 3) == r(4 * n) + 16 * n + tiles  # 12 bytes -> 16-byte records
    assert f(n, 9) == r(4 * n) + 64 * n + tiles  # 36 bytes -> 64-byte records
    assert f(n, 17) == r(4 * n) + 128 * n + tiles
    assert f(n, 18) == 0 and f(n, -1) == 0 and f(-1, 0) == 0 and f(1 << 31, 0) == 0
    assert f(0, 0) == f(1, 0) > 0


def _err(abm):
    return abm.lib().abm_last_error().decode()


def test_invalid_arguments_rejected_on_host(abm):
    L = abm.lib()
    soa = abm.Soa()
    rec = abm.Records()
    # NULL collection
    assert L.abm_select_update(None, None, C.byref(rec), None, None, None, None, 0, None) == \
        abm.ABM_E_INVALID
    assert "NULL" in _err(abm)
    # attribute count out of range
    soa.n_attrs, soa.capacity = 17, 10
    assert L.abm_select_update(C.byref(soa), None, C.byref(rec), None, None, None, None, 0,
                               None) == abm.ABM_E_INVALID
    # mismatched record attribute count
    soa.n_attrs, soa.capacity = 2, 0
    rec.n_attrs, rec.count = 3, 0
    assert L.abm_select_update(C.byref(soa), None, C.byref(rec), None, None, None, None, 0,
                               None) == abm.ABM_E_INVALID
    assert "differ" in _err(abm)
    # capacity beyond 2^31
    soa.n_attrs, soa.capacity, rec.n_attrs = 1, 1 << 31, 1
    assert L.abm_add_agents(C.byref(soa), C.byref(rec), None, None, None, 0, None) == \
        abm.ABM_E_INVALID
    # add_agents needs alive
    soa.capacity = 5
    soa.attr[0] = 16
    assert L.abm_add_agents(C.byref(soa), C.byref(rec), None, None, None, 0, None) == \
        abm.ABM_E_INVALID
    assert "alive" in _err(abm)
    # remove: misaligned mask
    soa.alive = 256
    assert L.abm_remove_agents(C.byref(soa), C.c_void_p(3), C.c_void_p(256), None, 0, None) == \
        abm.ABM_E_INVALID
    assert "aligned" in _err(abm)
    # resolve: negative sizes
    assert L.abm_resolve_conflicts(-1, None, None, None, 4, None, None, None, None) == \
        abm.ABM_E_INVALID
    assert L.abm_resolve_conflicts(4, None, None, None, 4, None, None, None, None) == \
        abm.ABM_E_INVALID
    # resolve: claim indices must fit winner[]'s int32 (2^31 claims is one too many)
    p = C.c_void_p(256)
    assert L.abm_resolve_conflicts(1 << 31, p, p, None, 4, p, p, p, None) == abm.ABM_E_INVALID
    assert "2^31" in _err(abm)
    # captured rollouts: no handle slot, bad chunking, NULL handles
    h = C.c_void_p()
    assert L.abm_predation_batched_graph(None, None, 10, 1, None, None, 0, None) == \
        abm.ABM_E_INVALID
    b = abm.Batch()
    assert L.abm_predation_batched_graph(C.byref(b), None, 0, 1, None, None, 0, C.byref(h)) == \
        abm.ABM_E_INVALID and not h.value
    assert L.abm_graph_replay(None, None) == abm.ABM_E_INVALID
    assert L.abm_graph_destroy(None) == abm.ABM_OK
    # select_indices: missing count
    assert L.abm_select_indices(None, 0, None, None, None, 0, None) == abm.ABM_E_INVALID
    # workspace init with nothing
    assert L.abm_workspace_init(None, 0, None) == abm.ABM_E_WORKSPACE


def test_invalid_predation_params_rejected_on_host(abm):
    L = abm.lib()
    st = abm.PredationStatePtrs()
    for bad in (dict(W=0), dict(R=0), dict(cap_s=0), dict(n_s0=5000), dict(gain_w=-1),
                dict(W=1 << 16, H=1 << 16)):
        p = abm.predation_params(**bad)
        assert L.abm_predation_init(C.byref(p), C.byref(st), None) == abm.ABM_E_INVALID, bad
    p = abm.predation_params()
    # NULL state arrays
    assert L.abm_predation_step(C.byref(p), C.byref(st), 1, None, 0, None) == abm.ABM_E_INVALID
    assert L.abm_predation_step(C.byref(p), None, 1, None, 0, None) == abm.ABM_E_INVALID


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    """No CPU fallback: a missing libabm.so is an ImportError at first use."""
    import paper_2508_16508_amd as pkg
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        pkg.lib()


def test_struct_layouts_match_header(abm, tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets
    (compiled with the host C compiler against include/abm.h)."""
    import ctypes as C
    structs = {"abm_soa": abm.Soa, "abm_records": abm.Records,
               "abm_predation_params": abm.PredationParams, "abm_species": abm.SpeciesPtrs,
               "abm_predation_state": abm.PredationStatePtrs, "abm_model_desc": abm.ModelDesc,
               "abm_batch": abm.Batch, "abm_tuning": abm.Tuning,
               "abm_traffic_params": abm.TrafficParams, "abm_traffic_state": abm.TrafficStatePtrs,
               "abm_lob_params": abm.LobParams, "abm_lob_state": abm.LobStatePtrs}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "abm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.splitlines():
        cname, field, val = line.split()
        py = structs[cname]
        if field == "size":
            assert C.sizeof(py) == int(val), cname
        else:
            assert getattr(py, field).offset == int(val), (cname, field)
