"""Autotuner for the persistent kernel.

For one workload (a batch of prefixes of order N with flags) it times the
counting launch on the GPU under every combination of

* fill-order variant (`dls_order_variant`: the Sec. 2.3 rule and variants of
  its weights and tie-breaks; the order changes the work, never the count),
* workgroup size,
* refill cadence (DFS steps between queue visits) and trigger (idle lanes
  that make a wave refill), grid size, smallest static chunk, mask layout,

checks that every candidate returns the same counts (tuning cannot change a
result), and keeps the fastest.  `tune_depth` does the same over split
depths for a split workload (the split is host work; only the GPU launch is
timed).  Results go to a JSON cache keyed by GPU architecture, order, flags
and a workload name, read back by `best()`.

    python -m paper_1709_02599_amd.autotune        # tunes the order-8 workload
"""
from __future__ import annotations

import itertools
import json
import os
import time
from typing import Dict, Iterable, List, Optional

import numpy as np

from . import (DLS_PLAIN, DLS_SYMBREAK, DlsLaunch, dls_count_async_ex, dls_kernel_time_ms, dls_split)

# DLS_AUTOTUNE_CACHE overrides the cache file (e.g. to tune into a scratch copy)
CACHE = os.environ.get("DLS_AUTOTUNE_CACHE") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                              "autotune_cache.json")
VARIANTS = tuple(range(8))
BLOCKS = (128, 256, 512)
REFILLS = (16, 32, 64)


def _arch(torch) -> str:
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(cache: dict) -> None:
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def key(arch: str, n: int, flags: int, workload: str) -> str:
    return f"{arch}:{n}:{flags}:{workload}"


def best(n: int, flags: int, workload: str, arch: Optional[str] = None) -> Optional[dict]:
    """Tuned launch settings for a workload, or None if never tuned."""
    cache = _load()
    if arch is None:
        import torch
        arch = _arch(torch)
    entry = cache.get(key(arch, n, flags, workload))
    return entry["best"] if entry else None


FIELDS = ("block", "blocks_per_cu", "steal_depth", "refill_every", "order_variant", "time_kernel",
          "expand_target", "chunk_min", "lds_masks", "refill_min", "wg_pool")


def _launch(settings: dict, time_kernel: int = 0) -> DlsLaunch:
    kw = {k: int(settings.get(k, 0)) for k in FIELDS}
    kw["time_kernel"] = time_kernel
    return DlsLaunch(**kw)


def time_launch(n: int, flags: int, pattern, d_pre, num: int, d_cnt, d_st, stream, settings: dict,
                reps: int = 3):
    """Mean duration (ms) of the search kernels over `reps` launches, measured
    by the library's event pairs on the launch stream, plus a digest of the
    counts of the last launch and the device status."""
    import torch
    dls_count_async_ex(n, flags, pattern, d_pre, num, d_cnt, d_st, stream, _launch(settings))  # warm-up
    timed = _launch(settings, 1)
    for _ in range(reps):
        dls_count_async_ex(n, flags, pattern, d_pre, num, d_cnt, d_st, stream, timed)
    torch.cuda.synchronize()
    ms, k = dls_kernel_time_ms(stream)
    assert k == reps
    c = d_cnt[:num]
    digest = (int(c.sum().item()), int((c * torch.arange(1, num + 1, device=c.device)).sum().item()))
    return ms, digest, int(d_st.item())


def tune(n: int, flags: int, prefixes: np.ndarray, workload: str, space: Optional[Dict[str, Iterable]] = None,
         default: Optional[dict] = None, reps: int = 3, save: bool = True, verbose: bool = True,
         plain: bool = True) -> dict:
    """Time every combination of the launch settings in `space` (field ->
    candidate values); all must give identical counts.  Keeps the fastest.
    plain: also time the plain kernel for reference (slow on big subtrees)."""
    import torch
    space = space or {"order_variant": VARIANTS, "block": BLOCKS, "refill_every": REFILLS}
    default = default or {"order_variant": 0, "block": 256, "refill_every": 32}
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    pre = np.ascontiguousarray(prefixes, dtype=np.uint8)
    num = len(pre)
    pattern = (pre[0] != 0xFF).astype(np.uint8)
    d_pre = torch.from_numpy(pre).to(dev)
    d_cnt = torch.zeros(num, dtype=torch.int64, device=dev)
    d_st = torch.zeros(1, dtype=torch.int32, device=dev)
    keys = list(space)
    table: List[dict] = []
    ref = None
    for values in itertools.product(*(space[k] for k in keys)):
        settings = dict(zip(keys, values))
        ms, digest, st = time_launch(n, flags, pattern, d_pre, num, d_cnt, d_st, stream, settings, reps)
        if st:
            raise RuntimeError(f"device status {st} for {settings}")
        if ref is None:
            ref = digest
        elif digest != ref:
            raise RuntimeError(f"counts differ for {settings}")
        table.append({**settings, "ms": ms})
        if verbose:
            print(f"  {settings}: {ms:.3f} ms", flush=True)
    # the plain kernel under the paper's order, for reference
    plain_ms = None
    if plain:
        plain_ms, digest, _ = time_launch(n, flags | DLS_PLAIN, pattern, d_pre, num, d_cnt, d_st, stream,
                                          {"block": 256}, reps)
        if digest != ref:
            raise RuntimeError("plain kernel counts differ")
    table.sort(key=lambda r: r["ms"])
    dflt = [r for r in table if all(r.get(k) == v for k, v in default.items())]
    result = {"best": table[0], "default": dflt[0] if dflt else None, "plain_ms": plain_ms,
              "candidates": len(table), "table": table[:12], "prefixes": num,
              "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    if save:
        cache = _load()
        cache[key(_arch(torch), n, flags, workload)] = result
        _save(cache)
    return result


def tune_depth(n: int, flags: int, depths: Iterable[int], workload: str, launch: Optional[dict] = None,
               reps: int = 3, save: bool = True) -> dict:
    """Time the counting launch for the split at each depth (same launch
    settings); the weighted totals must agree."""
    import torch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    total_ref = None
    for depth in depths:
        t0 = time.perf_counter()
        pre, mult = dls_split(n, flags, depth)
        split_s = time.perf_counter() - t0
        num = len(pre)
        pattern = (pre[0] != 0xFF).astype(np.uint8)
        d_pre = torch.from_numpy(pre).to(dev)
        d_cnt = torch.zeros(num, dtype=torch.int64, device=dev)
        d_st = torch.zeros(1, dtype=torch.int32, device=dev)
        kflags = flags & ~DLS_SYMBREAK & 1
        ms, _, st = time_launch(n, kflags, pattern, d_pre, num, d_cnt, d_st, stream, launch or {}, reps)
        tot = int((d_cnt * torch.from_numpy(mult.astype(np.int64)).to(dev)).sum().item())
        if total_ref is None:
            total_ref = tot
        elif tot != total_ref or st:
            raise RuntimeError(f"weighted total differs at depth {depth}")
        rows.append({"depth": depth, "prefixes": num, "ms": ms, "split_s": split_s})
    rows.sort(key=lambda r: r["ms"])
    result = {"best": rows[0], "table": rows, "weighted_total": total_ref}
    if save:
        cache = _load()
        cache[key(_arch(torch), n, flags, workload + ":depth")] = result
        _save(cache)
    return result


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--only", default="", help="comma-separated workload names")
    args = ap.parse_args(argv)
    only = set(filter(None, args.only.split(",")))

    def want(name):
        return not only or name in only

    if want("order8-symbreak-row1"):
        pre, mult = dls_split(8, DLS_SYMBREAK, 26)
        # stage 1: fill order, workgroup, refill cadence, mask layout
        r = tune(8, 0, pre, "order8-symbreak-row1", reps=args.reps,
                 space={"order_variant": VARIANTS, "block": BLOCKS, "refill_every": REFILLS, "lds_masks": (-1, 1)},
                 default={"order_variant": 0, "block": 256, "refill_every": 32, "lds_masks": -1}, save=False)
        first = {k: v for k, v in r["best"].items() if k != "ms"}
        # stage 2: grid size (1x to 4x the resident default; waves beyond
        # the resident ones only shrink the guided chunks), smallest chunk and
        # the number of idle lanes that triggers a refill
        d = 2048 // first["block"]
        r = tune(8, 0, pre, "order8-symbreak-row1", reps=args.reps,
                 space={**{k: (v,) for k, v in first.items()}, "blocks_per_cu": (0, d * 2, d * 3, d * 4),
                        "chunk_min": (0, 4, 16, 64), "refill_min": (1, 2, 4, 8, 16)},
                 default={"order_variant": 0, "block": 256, "refill_every": 32, "lds_masks": -1}, save=False)
        second = {k: v for k, v in r["best"].items() if k != "ms"}
        # stage 3: refill cadence against the refill trigger
        r = tune(8, 0, pre, "order8-symbreak-row1", reps=args.reps,
                 space={**{k: (v,) for k, v in second.items() if k not in ("refill_every", "refill_min")},
                        "refill_every": (32, 64, 96, 128), "refill_min": (1, 2, 4, 8, 16, 32)},
                 default={"order_variant": 0, "block": 256, "refill_every": 32, "lds_masks": -1}, save=False)
        third = {k: v for k, v in r["best"].items() if k != "ms"}
        # stage 4: the workgroup pool of the tail (on / off) against the
        # workgroup size, grid and smallest chunk
        r = tune(8, 0, pre, "order8-symbreak-row1", reps=args.reps,
                 space={**{k: (v,) for k, v in third.items() if k not in ("block", "blocks_per_cu", "chunk_min")},
                        "wg_pool": (0, -1), "block": (256, 512), "blocks_per_cu": (0, 8, 16),
                        "chunk_min": (4, 16, 64)},
                 default={"order_variant": 0, "block": 256, "refill_every": 32, "lds_masks": -1})
        print(json.dumps({"workload": "order8-symbreak-row1", "best": r["best"], "default": r["default"],
                          "plain_ms": r["plain_ms"]}), flush=True)
        d = tune_depth(8, DLS_SYMBREAK, (20, 22, 24, 26, 27, 28), "order8-symbreak",
                       launch={k: v for k, v in r["best"].items() if k != "ms"},
                       reps=args.reps)
        print(json.dumps({"workload": "order8-symbreak", "depths": d["table"]}), flush=True)
    if want("order7-diag11"):
        # order 7 split at the diagonals: a batch far smaller than the lanes
        pre, _ = dls_split(7, 0, 11)
        r = tune(7, 0, pre, "order7-diag11",
                 space={"expand_target": (0, -1, 1 << 13, 1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18),
                        "chunk_min": (0, 1, 4, 16, 64), "refill_every": (0, 16)},
                 default={"expand_target": 0, "chunk_min": 0, "refill_every": 0}, reps=args.reps)
        print(json.dumps({"workload": "order7-diag11", "best": r["best"], "plain_ms": r["plain_ms"],
                          "top": r["table"][:6]}), flush=True)
    if want("order8-diag14"):
        spre, _ = dls_split(8, 0, 14)
        s = tune(8, 0, spre, "order8-diag14",
                 space={"order_variant": (1, 5), "refill_every": (64, 128), "block": (256, 512),
                        "blocks_per_cu": (0, 8, 16), "refill_min": (1, 2, 4), "chunk_min": (16,),
                        "wg_pool": (0, -1)},
                 default={"order_variant": 0, "refill_every": 32, "blocks_per_cu": 0, "refill_min": 8,
                          "chunk_min": 0}, reps=1)
        print(json.dumps({"workload": "order8-diag14", "best": s["best"], "default": s["default"]}), flush=True)

    if want("order9-sample"):
        # 1 500 seeded workunits of the order-9 hourglass split (the full
        # count's workload); fullcount.py takes its launch from this entry
        import sys
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        import dls_workloads
        p9, _ = dls_split(9, DLS_SYMBREAK, 22)
        pos = np.array(dls_workloads.sample_positions(len(p9), 1500, seed=7), dtype=np.int64)
        s = tune(9, 0, np.ascontiguousarray(p9[pos]), "order9-sample",
                 space={"order_variant": (0, 2, 5), "refill_every": (32, 64, 128), "lds_masks": (0, -1),
                        "wg_pool": (0, -1)},
                 default={"order_variant": 0, "refill_every": 32}, reps=1, plain=False)
        print(json.dumps({"workload": "order9-sample", "best": s["best"], "default": s["default"]}), flush=True)


if __name__ == "__main__":
    main()
