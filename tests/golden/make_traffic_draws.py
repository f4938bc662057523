"""Print the random draws of the hand-worked traffic case (traffic_hand_L4.txt).

Calls only the oracle's RNG (pinned to the published SplitMix64 vectors):
lights and spawns are drawn per lane, lane changes per car slot.

    python tests/golden/make_traffic_draws.py
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle as O  # noqa: E402

LIGHT, LANE, SPAWN = 0x30, 0x31, 0x32


def dump(seed, steps, slots):
    for t in steps:
        for lane in range(3):
            h = O.rng(seed, t, lane, LIGHT)
            print(f"t={t} lane {lane} LIGHT = {h} green={h < 2 ** 31}")
        for i in range(slots):
            h = O.rng(seed, t, i, LANE)
            print(f"t={t} slot {i} LANE = {h} dl={O.uniform(h, 3) - 1}")
        for lane in range(3):
            h = O.rng(seed, t, lane, SPAWN)
            print(f"t={t} lane {lane} SPAWN = {h} spawn={h < 2 ** 31}")


if __name__ == "__main__":
    dump(9, range(4, 8), 7)
