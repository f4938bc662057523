"""abm_select_update_noalloc (no workspace, static scan state) against
abm_select_update on the same inputs: two calls in a row, the second on a
smaller input, both through the C ABI; plus its host-side size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2508_16508_amd import workloads as W


def _call_noalloc(abm, attrs, mask, recs):
    dst, upd = abm.make_soa(attrs), abm.make_records(recs)
    cnt = torch.full((3,), -7, dtype=torch.int64, device="cuda")
    rc = abm.lib().abm_select_update_noalloc(
        C.byref(dst), C.c_void_p(mask.data_ptr()), C.byref(upd), C.c_void_p(cnt[0:].data_ptr()),
        C.c_void_p(cnt[1:].data_ptr()), C.c_void_p(cnt[2:].data_ptr()),
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == abm.ABM_OK, abm.lib().abm_last_error()
    return cnt


def _call_ws(abm, attrs, mask, recs):
    dst, upd = abm.make_soa(attrs), abm.make_records(recs)
    ws = abm.workspace(max(dst.capacity, upd.count), abm.ABM_OP_SELECT_UPDATE)
    cnt = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    rc = abm.lib().abm_select_update(
        C.byref(dst), C.c_void_p(mask.data_ptr()), C.byref(upd), None,
        C.c_void_p(cnt[0:].data_ptr()), C.c_void_p(cnt[1:].data_ptr()), C.c_void_p(ws.data_ptr()),
        ws.numel(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == abm.ABM_OK, abm.lib().abm_last_error()
    return cnt, ws


@pytest.mark.gpu
def test_noalloc_matches_select_update_twice(abm):
    cases = [  # (seed, p, n, A, record fraction): the full microbenchmark, then smaller
        (3, 0.05, 1 << 24, 8, 1.0),
        (4, 0.5, 100_003, 3, 0.6),
    ]
    for seed, p, n, A, frac in cases:
        attrs = W.int32_rows(seed, A, n)
        mask = torch.from_numpy(W.bernoulli_mask(seed, p, n)).cuda()
        k = int(mask.sum().item())
        recs = torch.from_numpy(W.int32_rows(seed + 50, A, int(frac * k))).cuda()
        a = torch.from_numpy(attrs).cuda()
        b = a.clone()
        cnt = _call_noalloc(abm, a, mask, recs)
        ref, ws = _call_ws(abm, b, mask, recs)
        torch.cuda.synchronize()
        c, r = cnt.cpu().tolist(), ref.cpu().tolist()
        assert c[:2] == r == [min(k, recs.shape[1]), recs.shape[1] - min(k, recs.shape[1])]
        assert c[2] == 0 and abm.workspace_error(ws) == 0
        assert torch.equal(a, b), (seed, p, n)


def test_noalloc_rejects_capacity_above_its_maximum(abm):
    """2^28 + 1 slots: rejected on the host before any launch."""
    soa = abm.Soa()
    soa.n_attrs, soa.capacity = 1, (1 << 28) + 1
    soa.attr[0] = 256
    rec = abm.Records()
    rec.n_attrs, rec.count = 1, 0
    cnt = C.c_void_p(256)
    rc = abm.lib().abm_select_update_noalloc(C.byref(soa), C.c_void_p(256), C.byref(rec), cnt,
                                             None, None, None)
    assert rc == abm.ABM_E_INVALID
    assert b"2^28" in abm.lib().abm_last_error()
