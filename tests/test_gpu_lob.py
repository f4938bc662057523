"""GPU parity of the limit order books with batch matching (Sec. 5.3)
against the CPU oracle: every book of a batch must match the oracle run alone
with its own seed (seed + book), slot by slot, in its last price and in every
per-step statistic."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _run(abm, n_books, chunks, **kw):
    books = abm.OrderBooks(abm.lob_params(**kw), n_books)
    books.init()
    parts = []
    for c in chunks:
        s = torch.zeros((c, n_books, 8), dtype=torch.int64, device="cuda")
        books.run(c, s)
        parts.append(s)
    torch.cuda.synchronize()
    return books, torch.cat(parts).cpu().numpy()


def _check(abm, orc, books, st, steps, which=None):
    P = books.params
    host = {f: books.orders[f].cpu().numpy() for f in abm.LOB_FIELDS}
    last = books.last_price.cpu().numpy()
    assert abm.LOB_STAT_NAMES == orc.LOB_STATS
    for b in (which if which is not None else range(books.n_books)):
        kw = {f: getattr(P, f) for f, _ in P._fields_}
        kw["seed"] = (P.seed + b) & 0xFFFFFFFF
        OP = orc.lob_params(**kw)
        S = orc.lob_init(OP)
        exp = np.array([[d[k] for k in orc.LOB_STATS] for d in orc.lob_run(OP, S, steps)])
        assert np.array_equal(st[:, b], exp), f"stats of book {b}"
        assert last[b] == S.last_price, f"price of book {b}"
        for f in abm.LOB_FIELDS:
            assert np.array_equal(host[f][b], S.orders[f]), f"{f} of book {b}"


@pytest.mark.parametrize("n_books,kw", [
    (24, dict(cap=1000, traders=10, seed=0)),
    (16, dict(cap=50, traders=100, spread=5, expiry=6, seed=3)),            # full books, drops
    (8, dict(cap=1024, traders=1024, spread=200, max_qty=1 << 20, expiry=30, seed=5)),
    (6, dict(cap=1, traders=3, T_order=2 ** 32 - 1, seed=9)),
    (5, dict(cap=64, traders=0, seed=2)),
    (4, dict(cap=300, traders=40, spread=0, price0=1, seed=12)),           # prices pinned at the floor
])
def test_books_match_oracle(abm, orc, n_books, kw):
    books, st = _run(abm, n_books, (30, 1, 19), **kw)
    assert books.step == 50
    _check(abm, orc, books, st, 50)


def test_table4_scale_sample(abm, orc):
    """500 books of 1000 slots, 100 traders each, 100 steps (the shape of the
    paper's largest finance run): 10 books compared in full."""
    books, st = _run(abm, 500, (100,), cap=1000, traders=100, seed=40)
    _check(abm, orc, books, st, 100, which=range(0, 500, 51))


def test_invalid_arguments_are_rejected(abm):
    for kw in (dict(cap=0), dict(cap=1025), dict(traders=1025), dict(max_qty=0), dict(expiry=0),
               dict(price0=0)):
        books = abm.OrderBooks(abm.lob_params(cap=8), 1)
        books.params = abm.lob_params(**{"cap": 8, **kw})
        with pytest.raises(abm.AbmError):
            books.init()
