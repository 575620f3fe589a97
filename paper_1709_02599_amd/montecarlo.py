"""Monte Carlo estimate of the number of DLS of order N (Sec. 5.3).

The incomplete squares DLS_N^k have the first row fixed to 0..N-1 and the
first k cells in row-major order assigned so that no row, column or diagonal
repeats a value.  Their number N_N^k is counted exactly on the GPU
(`dls_count_cells`).  Every DLS extends exactly one DLS_N^k, so

    T_fixed(N) = N_N^k * E[completions of a uniformly drawn DLS_N^k],

and the mean over a uniform random sample estimates the expectation.

The sample is drawn exactly uniformly (a plain random walk over the cells
would favour squares with few siblings): the cells N..k-1 are cut into
stages; at each stage the extensions of the current square over the stage's
cells are enumerated on the host (`dls_split_cells`), weighted by their exact
numbers of extensions to all k cells (counted on the GPU), and one is drawn
with probability proportional to its weight.  The drawn squares' completions
to full squares are then counted on the GPU in one batch.

    python -m paper_1709_02599_amd.montecarlo --n 10 --k 32 --samples 64
"""
from __future__ import annotations

import math
import time
from typing import List, Optional, Sequence

import numpy as np

from . import dls_count_async_ex, dls_count_cells, dls_split_cells

EMPTY = 0xFF


def identity_prefix(n: int) -> np.ndarray:
    sq = np.full(n * n, EMPTY, dtype=np.uint8)
    sq[:n] = np.arange(n, dtype=np.uint8)
    return sq


def stages_for(n: int, k: int, first: Optional[int] = None) -> List[List[int]]:
    """Cells N..k-1 cut into stages: row 1 (or `first` cells), then chunks of
    at most 6 cells."""
    cells = list(range(n, k))
    if not cells:
        return []
    head = min(len(cells), first if first is not None else n)
    out = [cells[:head]]
    rest = cells[head:]
    while rest:
        out.append(rest[:6])
        rest = rest[6:]
    return out


class Sampler:
    """Exactly uniform draws of DLS_N^k (first row fixed, cells N..k-1
    row-major)."""

    def __init__(self, n: int, k: int, stages: Optional[Sequence[Sequence[int]]] = None):
        self.n, self.k = n, k
        self.stages = [list(s) for s in (stages or stages_for(n, k))]
        self.base = identity_prefix(n)
        # first stage: its extensions and their weights are shared by all draws
        tail = [c for s in self.stages[1:] for c in s]
        self.first = dls_split_cells(n, 0, self.base, self.stages[0]) if self.stages else self.base[None]
        self.first_w = (dls_count_cells(n, 0, tail, self.first) if self.stages
                        else np.ones(1, dtype=np.uint64))
        self.total = int(self.first_w.astype(object).sum())   # N_N^k

    @staticmethod
    def _pick(weights: np.ndarray, u: float) -> int:
        cum = np.cumsum(weights.astype(np.float64))
        # u * total as an integer position, then the bucket holding it
        pos = math.floor(u * float(cum[-1]))
        return int(np.searchsorted(cum, pos, side="right"))

    def draw(self, rng) -> np.ndarray:
        if self.total == 0:
            raise ValueError("no incomplete square to draw from")
        sq = self.first[self._pick(self.first_w, rng.uniform())]
        for t in range(1, len(self.stages)):
            ext = dls_split_cells(self.n, 0, sq, self.stages[t])
            tail = [c for s in self.stages[t + 1:] for c in s]
            w = dls_count_cells(self.n, 0, tail, ext) if tail else np.ones(len(ext), dtype=np.uint64)
            sq = ext[self._pick(w, rng.uniform())]
        return sq.copy()


def completions(n: int, squares: np.ndarray, launch=None) -> np.ndarray:
    """Number of full DLS extending each square (one GPU batch; the squares
    must assign the same cells)."""
    import torch
    sq = np.ascontiguousarray(squares, dtype=np.uint8).reshape(-1, n * n)
    dev = torch.device("cuda:0")
    d_pre = torch.from_numpy(sq).to(dev)
    d_cnt = torch.zeros(len(sq), dtype=torch.int64, device=dev)
    d_st = torch.zeros(1, dtype=torch.int32, device=dev)
    pattern = (sq[0] != EMPTY).astype(np.uint8)
    dls_count_async_ex(n, 0, pattern, d_pre, len(sq), d_cnt, d_st, None, launch)
    torch.cuda.synchronize()
    if int(d_st.item()):
        raise RuntimeError(f"device status {int(d_st.item())}")
    return d_cnt.cpu().numpy().view(np.uint64).copy()


def estimate(n: int, k: int, samples: int, rng, launch=None, batch: Optional[int] = None, log=None) -> dict:
    """Draw `samples` squares and count their completions, `batch` at a time
    (all at once by default); `log` receives a progress line per batch.  The
    draws depend only on the generator, not on the batching."""
    t0 = time.perf_counter()
    s = Sampler(n, k)
    t1 = time.perf_counter()
    batch = batch or samples
    parts, draw_s, count_s = [], 0.0, 0.0
    for b0 in range(0, samples, batch):
        ta = time.perf_counter()
        drawn = np.stack([s.draw(rng) for _ in range(min(batch, samples - b0))])
        tb = time.perf_counter()
        parts.append(completions(n, drawn, launch))
        tc = time.perf_counter()
        draw_s += tb - ta
        count_s += tc - tb
        if log:
            done = np.concatenate(parts).astype(np.float64)
            log(f"{len(done)}/{samples} samples: mean completions {done.mean():.4e}, "
                f"estimate {s.total * done.mean():.4e}, batch {tc - ta:.1f} s")
    c = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)
    x = c.astype(np.float64)
    mean = float(x.mean())
    se = float(x.std(ddof=1) / math.sqrt(len(x))) if len(x) > 1 else float("nan")
    return {"n": n, "k": k, "N_k": s.total, "samples": samples, "mean_completions": mean,
            "estimate": s.total * mean, "std_error": s.total * se, "squares_counted": int(c.sum()),
            "seconds": {"count_N_k": t1 - t0, "draw": draw_s, "complete": count_s},
            "completions": [int(v) for v in c]}


def main(argv=None):
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import dls_workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--samples", type=int, default=64)
    ap.add_argument("--seed", type=int, default=dls_workloads.DEFAULT_SEED)
    ap.add_argument("--batch", type=int, default=16, help="samples counted per GPU batch")
    args = ap.parse_args(argv)
    r = estimate(args.n, args.k, args.samples, dls_workloads.SplitMix64(args.seed), batch=args.batch,
                 log=lambda line: print(line, flush=True))
    r.pop("completions")
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
