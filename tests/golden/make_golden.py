"""Writes oracle_distances.json: distances of the stand-in workloads computed
by the CPU oracle only (its Brouwer-Zimmermann over the F4 construction),
and for config 3 the oracle's round-by-round trace (the combinations its
BZ enumerates to reach the exact distance).
Run from the repository root:
    python tests/golden/make_golden.py [config2] [config3] [config4]
With no argument every part is (re)computed; with arguments only those
parts are, and the others are kept from the existing file.

The config-4 sample is a fixed list of draw indices of the config-4 batch
(n 28..80, both fields), spread over predicted work from 1e4 to 1e11
combinations and including codes whose F4 matrices get two-row caps; the
indices are inputs chosen by hand, the distances come from the oracle.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2408_10743_amd import workloads as W  # noqa: E402

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_distances.json")

# Draw indices of W.config4(800): additive (even) and F4-linear (odd).
CONFIG4_SAMPLE = [4, 30, 60, 8, 6, 82, 52, 116, 22, 0, 164, 44, 88, 176, 538, 556, 100, 64,
                  19, 7, 25, 595, 65, 15, 43, 13, 63, 37, 3, 587, 219, 613, 629, 483]


def part_config2(out):
    out["config2"] = []
    for i in range(20):
        G, f = W.config2(i)
        d, _, _ = O.bz(O.expand(G, f), O.DIAG_F4, 8)
        out["config2"].append(d)
        print("config2", i, d, flush=True)


def part_config3(out):
    out["config3"] = []
    out["config3_oracle_rounds"] = []
    for i in range(5):
        t0 = time.time()
        G, f = W.config3(i)
        d, _, log = O.bz(O.expand(G, f), O.DIAG_F4, 2)
        out["config3"].append(d)
        # the oracle's BZ trace: (t, j, L, U, combinations) after each round
        out["config3_oracle_rounds"].append([list(r) for r in log])
        print("config3", i, d, f"{time.time() - t0:.1f}s", log[-1], flush=True)


def part_config4(out):
    pool = W.config4(800)
    rows = []
    for i in CONFIG4_SAMPLE:
        t0 = time.time()
        G, f = pool[i]
        n = G.shape[1] // 2 if f == 2 else G.shape[1]
        d, _, log = O.bz(O.expand(G, f), O.DIAG_F4, 8)
        visited = sum(r[4] for r in log)
        rows.append({"index": i, "n": n, "m": int(G.shape[0]), "field": f, "d": d,
                     "oracle_combinations": visited})
        print("config4", i, n, f, d, visited, f"{time.time() - t0:.1f}s", flush=True)
    out["config4_sample"] = rows


def main():
    parts = sys.argv[1:] or ["config2", "config3", "config4"]
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    out["_source"] = "CPU oracle (oracle/qdo.c) on paper_2408_10743_amd/workloads.py inputs"
    for p in parts:
        {"config2": part_config2, "config3": part_config3, "config4": part_config4}[p](out)
        json.dump(out, open(PATH, "w"), indent=1)
    print("wrote", PATH)


if __name__ == "__main__":
    main()
