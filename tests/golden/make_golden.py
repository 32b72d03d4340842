"""Writes oracle_distances.json: distances of the stand-in workloads computed
by the CPU oracle only (brute force where the rank allows, else its
Brouwer-Zimmermann).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2408_10743_amd import workloads as W  # noqa: E402


def main():
    out = {"_source": "CPU oracle (oracle/qdo.c) on paper_2408_10743_amd/workloads.py inputs",
           "config2": [], "config3": []}
    for i in range(20):
        G, f = W.config2(i)
        d, _, _ = O.bz(O.expand(G, f), O.DIAG_F4, 8)
        out["config2"].append(d)
        print("config2", i, d, flush=True)
    for i in range(2):
        t0 = time.time()
        G, f = W.config3(i)
        d, _, log = O.bz(O.expand(G, f), O.DIAG_F4, 2)
        out["config3"].append(d)
        print("config3", i, d, f"{time.time() - t0:.1f}s", log[-1], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_distances.json")
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
