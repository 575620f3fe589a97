"""Readers for the text fixtures under tests/golden/ (each cites its source)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EMPTY = 0xFF


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line


def counts():
    """{(N, kind): value} from counts.txt."""
    out = {}
    for line in _lines("counts.txt"):
        n, kind, value = line.split()[:3]
        out[(int(n), kind)] = int(value)
    return out


def keyed(name):
    out = {}
    for line in _lines(name):
        k, v = line.split()
        out[k] = int(v)
    return out


def fig1_order():
    """Flat cell indices of the order-9 fill order, position 1 first."""
    rows = [line.split() for line in _lines("fig1_order_n9.txt")]
    pos = {}
    for i, r in enumerate(rows):
        for j, t in enumerate(r):
            if t != "-":
                pos[int(t)] = i * 9 + j
    return [pos[k] for k in sorted(pos)]


def fig2():
    """(left, right) order-10 designs of Fig. 2 as flat uint8 arrays."""
    blocks, cur = {}, None
    for line in _lines("fig2_hourglass_n10.txt"):
        if line in ("left", "right"):
            cur = blocks.setdefault(line, [])
            continue
        cur.extend(EMPTY if t == "_" else int(t) for t in line.split())
    return (np.array(blocks["left"], dtype=np.uint8), np.array(blocks["right"], dtype=np.uint8))


def vs10_sample():
    """The seeded VS order-10 sample written by make_vs10_sample.py:
    (total workunits, left cells, positions, prefixes [K, 100], counts)."""
    n = 10
    total, cells, pos, rows, counts = None, None, [], [], []
    for line in _lines("vs10_sample.txt"):
        t = line.split()
        if t[0] == "total":
            total = int(t[1])
        elif t[0] == "cells":
            cells = [int(x) for x in t[1:]]
        else:
            p, digits, c = int(t[0]), t[1], int(t[2])
            sq = np.full(n * n, EMPTY, dtype=np.uint8)
            sq[:n] = np.arange(n)
            for cell, d in zip(cells, digits):
                v = int(d, 16)
                i, j = divmod(cell, n)
                sq[cell] = v
                sq[i * n + (n - 1 - j)] = n - 1 - v
            pos.append(p)
            rows.append(sq)
            counts.append(c)
    return total, cells, np.array(pos, dtype=np.int64), np.stack(rows), np.array(counts, dtype=np.uint64)
