"""Writes the stored expected values under tests/golden/ by calling only the
oracle package (never the GPU library).

connected_counts.json : connected diagram counts with unit propagators and
    weight x per closed cycle (x = w * N), n = 1..12, from the exponential
    formula (oracle.counts): the full sum over all diagrams is the rising
    factorial x (x+1) ... (x+2n-1) and A = exp(C).
plan_counts.json : per-flavour state / extension / close / shift-edge / mask
    counts of the vertex-level DP (oracle.dp with counts=True), n = 1..12.

Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import counts  # noqa: E402


def main():
    xs = [1, 2, 3, -1, -2, -3, -4, -6]
    seqs = {str(x): [str(v) for v in counts.connected_counts(12, x)[1:]] for x in xs}
    with open(os.path.join(HERE, "connected_counts.json"), "w") as f:
        json.dump({"source": "oracle.counts.connected_counts (exponential formula, exact integers)",
                   "meaning": "c_n for n=1..12 with G=1 and weight x=w*N per closed cycle",
                   "sequences": seqs}, f, indent=1)
    out = {}
    for n in range(1, 13):
        _, c = oracle.dp(np.ones((n, n)), 2, 0, stub=np.zeros(1), counts=True, precision="d")
        out[str(n)] = c
        print(n, c, flush=True)
    with open(os.path.join(HERE, "plan_counts.json"), "w") as f:
        json.dump({"source": "oracle.dp(counts=True): per flavour slot, shifts enabled",
                   "counts": out}, f, indent=1)


if __name__ == "__main__":
    main()
