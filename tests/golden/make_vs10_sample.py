"""Writes vs10_sample.txt: a seeded uniform sample of 4096 workunits of the
vertically symmetric order-10 count (first row fixed; the first 17 left-half
cells of the fill order, each with its mirror) and the oracle's exact count of
each.  Calls only the oracle (and the seeded position generator).

    python tests/golden/make_vs10_sample.py        # about 5 minutes on 8 cores
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import dls_workloads  # noqa: E402

N, DEPTH, K, SEED = 10, 17, 4096, 170902599


def cells_with_mirrors(n, order):
    cells = []
    for c in order:
        cells.append(c)
        m = (c // n) * n + (n - 1 - c % n)
        if m != c:
            cells.append(m)
    return cells


def main():
    base = oracle.identity_prefix(N)
    left = oracle.fill_order(N, vs=True)[:DEPTH]
    cells = cells_with_mirrors(N, left)
    total = oracle.count_assignments(N, base, cells, vs=True)
    pos = dls_workloads.sample_positions(total, K, seed=SEED)
    pre = oracle.assignments_at(N, base, cells, pos, vs=True)
    counts = oracle.count_many(N, pre, vs=True)
    with open(os.path.join(HERE, "vs10_sample.txt"), "w") as f:
        f.write("# Vertically symmetric DLS of order 10 (Sec. 5.4), first row fixed.\n")
        f.write(f"# Split: the first {DEPTH} left-half cells of the fill order (Sec. 2.3), each\n")
        f.write(f"# with its mirror; {total} workunits.  Sample: {K} positions drawn by\n")
        f.write(f"# dls_workloads.sample_positions(total, {K}, seed={SEED}).  Counts by the oracle.\n")
        f.write("# Written by tests/golden/make_vs10_sample.py.\n")
        f.write("# line: position, values of the listed cells (hex digits), exact count\n")
        f.write("total %d\n" % total)
        f.write("cells %s\n" % " ".join(str(c) for c in left))
        for p, sq, c in zip(pos, pre, counts):
            digits = "".join("%x" % sq[cc] for cc in left)
            f.write("%d %s %d\n" % (p, digits, c))
    est = float(counts.mean()) * total
    print("estimate", est, "from", K, "prefixes")


if __name__ == "__main__":
    main()
