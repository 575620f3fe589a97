"""Seeded synthetic inputs: random numbers and random partial squares.

This module draws random numbers and builds inputs; it computes no counts.
Both the GPU path and the oracle receive the inputs it builds, so it is kept
apart from either.

* ``SplitMix64`` -- the counter-based generator of Steele, Lea and Flood
  (2014): state += 0x9E3779B97F4A7C15, then two xor-shift-multiply rounds.
* ``sample_positions`` -- k distinct positions in [0, P), uniform, sorted.
* ``random_permutations`` -- uniform permutations (Fisher-Yates), e.g. the
  order in which a search tries values when it builds a complete square;
  ``blank_cells`` -- a square with uniformly drawn cells emptied.
* ``random_job`` -- a serving request: order N, flags, and a prefix made of the
  identity first row plus k random cells, each a random empty cell given a
  random value that repeats no value already in its row, column or diagonal
  (for vertical symmetry, a left-half cell and its mirror).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

MASK64 = (1 << 64) - 1
EMPTY = 0xFF
DEFAULT_SEED = 170902599


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def below(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection (no modulo bias)."""
        if bound <= 0:
            raise ValueError("bound must be positive")
        limit = (1 << 64) - ((1 << 64) % bound)
        while True:
            x = self.next()
            if x < limit:
                return x % bound

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / (1 << 53))


def random_permutations(n: int, count: int, rng: SplitMix64) -> np.ndarray:
    """count uniform random permutations of 0..n-1 ([count, n] uint8,
    Fisher-Yates)."""
    out = np.zeros((count, n), dtype=np.uint8)
    for r in range(count):
        p = list(range(n))
        for t in range(n - 1, 0, -1):
            u = rng.below(t + 1)
            p[t], p[u] = p[u], p[t]
        out[r] = p
    return out


def blank_cells(n: int, square: np.ndarray, k: int, vs: bool, rng: SplitMix64) -> np.ndarray:
    """A copy of `square` with k uniformly drawn cells emptied (for vs, k
    left-half cells together with their mirrors)."""
    sq = np.array(square, dtype=np.uint8).reshape(n * n).copy()
    cand = [c for c in range(n * n) if not vs or 2 * (c % n) < n - 1]
    for pos in sample_positions(len(cand), min(k, len(cand)), seed=rng.next()):
        c = cand[int(pos)]
        sq[c] = EMPTY
        if vs:
            sq[(c // n) * n + n - 1 - c % n] = EMPTY
    return sq


def sample_positions(total: int, k: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """k distinct uniform positions in [0, total), sorted (Floyd's method)."""
    if k > total:
        raise ValueError("sample larger than population")
    rng = SplitMix64(seed)
    chosen = set()
    for j in range(total - k, total):
        t = rng.below(j + 1)
        chosen.add(t if t not in chosen else j)
    return np.array(sorted(chosen), dtype=np.int64)


@dataclass
class Job:
    jid: int
    n: int
    vs: bool
    prefix: np.ndarray          # n*n uint8
    k: int                      # cells added beyond the first row
    arrival: float              # seconds after the stream start


def _free_values(sq: np.ndarray, n: int, i: int, j: int) -> List[int]:
    a = sq.reshape(n, n)
    used = set(int(x) for x in a[i, :]) | set(int(x) for x in a[:, j])
    if i == j:
        used |= set(int(a[t, t]) for t in range(n))
    if i + j == n - 1:
        used |= set(int(a[t, n - 1 - t]) for t in range(n))
    return [v for v in range(n) if v not in used]


def random_prefix(n: int, k: int, vs: bool, rng: SplitMix64, max_tries: int = 1000) -> np.ndarray:
    """Identity first row plus k random cells (k counts both cells of a mirror
    pair for vs); a cell whose candidate list is empty is skipped and another
    one drawn."""
    sq = np.full(n * n, EMPTY, dtype=np.uint8)
    sq[:n] = np.arange(n, dtype=np.uint8)
    added = 0
    tries = 0
    while added < k and tries < max_tries:
        tries += 1
        empty = [c for c in range(n * n) if sq[c] == EMPTY and (not vs or 2 * (c % n) < n)]
        if not empty:
            break
        c = empty[rng.below(len(empty))]
        i, j = divmod(c, n)
        vals = _free_values(sq, n, i, j)
        if vs:
            jj = n - 1 - j
            ok = []
            for v in vals:
                sq[c] = v
                if jj != j and (n - 1 - v) in _free_values(sq, n, i, jj):
                    ok.append(v)
                sq[c] = EMPTY
            vals = ok
        if not vals:
            continue
        v = vals[rng.below(len(vals))]
        sq[c] = v
        added += 1
        if vs and n - 1 - j != j:
            sq[i * n + n - 1 - j] = n - 1 - v
            added += 1
    return sq


def job_stream(count: int, rate: float, seed: int = DEFAULT_SEED,
               orders=(7, 8, 9), vs_choices=(False, True),
               k_range: Optional[tuple] = None) -> List[Job]:
    """Poisson arrivals at `rate` jobs/s; N uniform over `orders`, flags
    uniform over plain/VS, k uniform in [N, 3N] (or `k_range`)."""
    rng = SplitMix64(seed)
    t = 0.0
    jobs = []
    for jid in range(count):
        u = rng.uniform()
        t += -np.log(1.0 - u) / rate
        n = orders[rng.below(len(orders))]
        vs = vs_choices[rng.below(len(vs_choices))]
        lo, hi = k_range if k_range else (n, 3 * n)
        k = lo + rng.below(hi - lo + 1)
        jobs.append(Job(jid, n, vs, random_prefix(n, k, vs, rng), k, t))
    return jobs
