"""Pins for the oracle's limit order books with batch matching (Sec. 5.3).

The paper matches many orders at once by sorting both sides by price and
taking cumulative sums of shares, and prints no trajectories.  The oracle's
batch rule is pinned against an independent serial matcher (repeatedly trade
the best bid against the best ask while they cross, in price-time priority),
the serial formulation the paper contrasts its matching with, on many
random books; by a book matched by hand; and by invariants of whole runs
(no crossed book after a step, volume conservation, expiry, capacity)."""
import numpy as np
import pytest

FIELDS = ("side", "price", "qty", "time", "alive")


def _book(orc, cap, orders, step, **kw):
    P = orc.lob_params(cap=cap, T_order=0, expiry=10 ** 6, **kw)
    S = orc.lob_init(P)
    for i, (side, price, qty, time) in enumerate(orders):
        for f, v in zip(FIELDS, (side, price, qty, time, 1)):
            S.orders[f][i] = v
    S.step = step
    return P, S


def _serial_match(S):
    """Best bid against best ask, one trade at a time, price-time priority."""
    o = {f: S.orders[f].copy() for f in FIELDS}
    live = [i for i in range(o["alive"].size) if o["alive"][i]]
    bids = sorted([i for i in live if o["side"][i] == 0], key=lambda i: (-o["price"][i], o["time"][i], i))
    asks = sorted([i for i in live if o["side"][i] == 1], key=lambda i: (o["price"][i], o["time"][i], i))
    rem = {i: int(o["qty"][i]) for i in live}
    vol, bi, ai, last = 0, 0, 0, None
    while bi < len(bids) and ai < len(asks) and o["price"][bids[bi]] >= o["price"][asks[ai]]:
        b, a = bids[bi], asks[ai]
        q = min(rem[b], rem[a])
        rem[b] -= q
        rem[a] -= q
        vol += q
        last = (int(o["price"][b]), int(o["price"][a]))
        if rem[b] == 0:
            bi += 1
        if rem[a] == 0:
            ai += 1
    return vol, rem, last


def test_hand_matched_book(orc):
    # slot: side, price, qty, time  -- buys 0..2, sells 3..5
    orders = [(0, 105, 3, 0), (0, 103, 5, 1), (0, 105, 2, 2),
              (1, 101, 4, 0), (1, 104, 3, 1), (1, 106, 5, 0)]
    P, S = _book(orc, 8, orders, step=2)
    st = orc.lob_step(P, S)
    # buys by priority: slot 0 (105, t0), slot 2 (105, t2), slot 1 (103): CB 3, 5, 10
    # sells: slot 3 (101), slot 4 (104), slot 5 (106): CS 4, 7, 12
    # V = max(min(3, 7), min(5, 7), min(10, 4)) = 5; the share-5 prices are 105 and 104
    assert st["volume"] == 5 and st["price"] == 104 and st["filled_orders"] == 4
    assert list(S.orders["alive"][:6]) == [0, 1, 0, 0, 1, 1]
    assert S.orders["qty"][4] == 2 and S.orders["qty"][1] == 5 and S.orders["qty"][5] == 5
    assert (st["buys"], st["sells"]) == (1, 2)


@pytest.mark.parametrize("n_orders,cap", [(2, 4), (10, 16), (60, 64), (300, 400)])
def test_batch_equals_serial_matcher(orc, n_orders, cap):
    g = np.random.default_rng(n_orders)
    for trial in range(150):
        orders = [(int(g.integers(0, 2)), int(g.integers(95, 106)), int(g.integers(1, 8)),
                   int(g.integers(0, 5))) for _ in range(n_orders)]
        P, S = _book(orc, cap, orders, step=5)
        vol, rem, last = _serial_match(S)
        st = orc.lob_step(P, S)
        assert st["volume"] == vol
        for i, q in rem.items():
            if q == 0:
                assert S.orders["alive"][i] == 0
            else:
                assert S.orders["alive"][i] == 1 and S.orders["qty"][i] == q
        if vol > 0:
            assert st["price"] == (last[0] + last[1]) // 2


def test_runs_keep_the_book_uncrossed(orc):
    for seed in range(20):
        P = orc.lob_params(cap=200, traders=25, spread=15, expiry=12, seed=seed)
        S = orc.lob_init(P)
        for t in range(60):
            active_before = int(S.orders["alive"].sum())
            st = orc.lob_step(P, S)
            o, live = S.orders, S.orders["alive"] != 0
            bids = o["price"][live & (o["side"] == 0)]
            asks = o["price"][live & (o["side"] == 1)]
            if bids.size and asks.size:
                assert bids.max() < asks.min()
            assert st["buys"] + st["sells"] == int(live.sum()) <= P.cap
            assert st["placed"] + st["dropped"] <= P.traders
            assert np.all(o["time"][live] > t - P.expiry)
            assert 1 <= st["price"] < 2 ** 24
            assert int(live.sum()) <= active_before - st["expired"] + st["placed"]


def test_full_book_drops_new_orders(orc):
    P = orc.lob_params(cap=5, traders=40, T_order=2 ** 32 - 1, spread=0, expiry=10 ** 6, seed=3)
    S = orc.lob_init(P)
    st = orc.lob_step(P, S)
    assert st["placed"] == 5 and st["dropped"] == 35


def test_no_orders_no_change(orc):
    P = orc.lob_params(cap=30, T_order=0, seed=1)
    S = orc.lob_init(P)
    for st in orc.lob_run(P, S, 10):
        assert st["placed"] == st["volume"] == 0 and st["price"] == P.price0
