"""Writes the stored walk-count fixture used by the oracle pins.

Calls only the oracle's brute-force walk enumerator.  Graph: a triangle
{0,1,2} with a tail 2-3-4, query node 0, walks of length 1..8.  Run:
python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import walk_counts  # noqa: E402

EDGES = [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]


def main():
    n = 5
    adj = [[] for _ in range(n)]
    for u, v in EDGES:
        adj[u].append(v)
        adj[v].append(u)
    rp = np.zeros(n + 1, np.int64)
    col = []
    for u in range(n):
        col += sorted(adj[u])
        rp[u + 1] = len(col)
    counts = walk_counts(n, rp, np.array(col), 0, 8)
    out = {"source": "oracle.walk_counts (brute-force enumeration of walks, eq. KatzPath)",
           "n": n, "edges": EDGES, "q": 0, "max_len": 8, "counts": counts}
    with open(os.path.join(HERE, "walks_tri_tail.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
