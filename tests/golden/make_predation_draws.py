"""Print the random draws used by the hand-worked predation cases.

The expected states in ``predation_hand_1x1.txt`` and ``predation_hand_3x3.txt``
were worked out by hand from these draws and the model rules (Sec. 5.1, with
the step order move, eat, breed, die, regrow); ``predation_multi_prey_1x1.txt``
from the prey and eat keys of one step; ``predation_moves_8dirs.txt`` from the
move draws of step 0 for seed 30, whose eight sheep draw all eight directions.
This script calls only the oracle's
RNG (which is itself pinned to the published SplitMix64 vectors).

    python tests/golden/make_predation_draws.py
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle as O  # noqa: E402

INIT = 0xFFFFFFFF
NAMES = {0x01: "GRASS_GROWN", 0x02: "GRASS_CD", 0x10: "S_X", 0x11: "S_Y", 0x12: "S_E",
         0x13: "S_MOVE", 0x14: "S_GRASS_KEY", 0x15: "S_PREY_KEY", 0x16: "S_BREED",
         0x20: "W_X", 0x21: "W_Y", 0x22: "W_E", 0x23: "W_MOVE", 0x24: "W_EAT_KEY",
         0x26: "W_BREED"}


def dump(seed, cells, cap_s, cap_w, steps):
    print(f"# seed={seed}")
    for c in range(cells):
        for p in (0x01, 0x02):
            print(f"INIT cell {c} {NAMES[p]} = {O.rng(seed, INIT, c, p)}")
    for i in range(cap_s):
        for p in (0x10, 0x11, 0x12):
            print(f"INIT sheep {i} {NAMES[p]} = {O.rng(seed, INIT, i, p)}")
    for i in range(cap_w):
        for p in (0x20, 0x21, 0x22):
            print(f"INIT wolf {i} {NAMES[p]} = {O.rng(seed, INIT, i, p)}")
    for t in range(steps):
        for i in range(cap_s):
            for p in (0x13, 0x14, 0x15, 0x16):
                h = O.rng(seed, t, i, p)
                extra = f" dir={h >> 29}" if p == 0x13 else ""
                print(f"t={t} sheep {i} {NAMES[p]} = {h}{extra}")
        for i in range(cap_w):
            for p in (0x23, 0x24, 0x26):
                h = O.rng(seed, t, i, p)
                extra = f" dir={h >> 29}" if p == 0x23 else ""
                print(f"t={t} wolf {i} {NAMES[p]} = {h}{extra}")


def dump_keys(seed, step, n_s, n_w):
    print(f"# seed={seed} step={step}")
    for i in range(n_s):
        print(f"t={step} sheep {i} S_PREY_KEY = {O.rng(seed, step, i, 0x15)}")
    for j in range(n_w):
        print(f"t={step} wolf {j} W_EAT_KEY = {O.rng(seed, step, j, 0x24)}")


def dump_moves(seed, step, n_s, n_w):
    print(f"# seed={seed} step={step}")
    for sp, n, p in (("sheep", n_s, 0x13), ("wolf", n_w, 0x23)):
        for i in range(n):
            h = O.rng(seed, step, i, p)
            print(f"t={step} {sp} {i} {NAMES[p]} = {h} dir={h >> 29}")


if __name__ == "__main__":
    dump(5, 1, 4, 2, 2)
    dump(11, 9, 3, 3, 2)
    dump_keys(21, 7, 4, 3)
    dump_moves(30, 0, 8, 8)
