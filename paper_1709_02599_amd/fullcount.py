"""Resumable full counts: a large count split into chunks that run as
separate processes (or on separate days), each writing its partial sum to a
file, and a merge step that checks the chunks fit together.

A chunk is the prefixes of dls_split(n, flags, depth) at positions
i, i + K, i + 2K, ... (chunk i of K): interleaving balances the uneven
subtrees of the depth-first split.  Within a chunk the prefixes are counted
in sub-batches, each one persistent-kernel launch, and the partial sum is
written after every sub-batch, so an interrupted chunk resumes where it
stopped.  With DLS_SYMBREAK the workunits are canonical hourglass designs and
the sum is sum(class power * count) (Corollary 1), i.e. the number of DLS
with the first row fixed.

    python -m paper_1709_02599_amd.fullcount --n 9 --symbreak --depth 22 \\
        --chunks 6 --chunk 0 --out counts9/
    python -m paper_1709_02599_amd.fullcount --merge counts9/
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

from . import DLS_SYMBREAK, DLS_VSYM, DlsLaunch, dls_count_async_ex, dls_kernel_time_ms, dls_split


def split_digest(pre: np.ndarray, mult: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pre).tobytes())
    h.update(np.ascontiguousarray(mult).tobytes())
    return h.hexdigest()


def load_split(n: int, flags: int, depth: int, cache: str | None = None):
    """dls_split(n, flags, depth), optionally through a cache file (plain
    .npz, no pickled objects) so that the chunks of one count split once.
    A cache whose recorded parameters or digest do not match is rebuilt."""
    if cache and os.path.exists(cache):
        with np.load(cache, allow_pickle=False) as z:
            if (int(z["n"]), int(z["flags"]), int(z["depth"])) == (n, flags, depth):
                pre, mult = z["pre"], z["mult"]
                if split_digest(pre, mult) == str(z["digest"]):
                    return pre, mult
    pre, mult = dls_split(n, flags, depth)
    if cache:
        tmp = cache + ".tmp.npz"
        np.savez(tmp, n=n, flags=flags, depth=depth, pre=pre, mult=mult, digest=split_digest(pre, mult))
        os.replace(tmp, cache)
    return pre, mult


def _path(out: str, chunk: int, chunks: int) -> str:
    return os.path.join(out, f"chunk_{chunk:04d}_of_{chunks:04d}.json")


def run_chunk(n: int, flags: int, depth: int, chunk: int, chunks: int, out: str, batches: int = 10,
              launch: dict | None = None, log=print, stop_after: int | None = None,
              split_cache: str | None = None) -> dict:
    """Count chunk `chunk` of `chunks`; resumes from the chunk file in `out`
    if one exists.  stop_after: return after that many batches of this call
    (the file records the progress).  split_cache: see load_split."""
    import torch
    os.makedirs(out, exist_ok=True)
    path = _path(out, chunk, chunks)
    t0 = time.perf_counter()
    pre, mult = load_split(n, flags, depth, split_cache)
    digest = split_digest(pre, mult)
    log(f"split: {len(pre)} workunits in {time.perf_counter() - t0:.1f} s, digest {digest[:16]}")
    state = {"n": n, "flags": flags, "depth": depth, "chunk": chunk, "chunks": chunks,
             "workunits": int(len(pre)), "split_digest": digest, "batches": batches, "done_batches": 0,
             "weighted_sum": "0", "squares": "0", "kernel_seconds": 0.0}
    if os.path.exists(path):
        with open(path) as f:
            prev = json.load(f)
        if prev.get("split_digest") != digest or prev.get("batches") != batches:
            raise RuntimeError(f"{path} belongs to another split or batching")
        state = prev
        log(f"resuming at batch {state['done_batches']} of {batches}")
    idx = np.arange(chunk, len(pre), chunks, dtype=np.int64)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    kflags = flags & DLS_VSYM
    lc = DlsLaunch(**{**(launch or {}), "time_kernel": 1})
    ran = 0
    for b in range(state["done_batches"], batches):
        if stop_after is not None and ran >= stop_after:
            break
        ran += 1
        sel = idx[b::batches]
        if len(sel) == 0:
            state["done_batches"] = b + 1
            continue
        sp = np.ascontiguousarray(pre[sel])
        d_pre = torch.from_numpy(sp).to(dev)
        d_cnt = torch.zeros(len(sel), dtype=torch.int64, device=dev)
        d_st = torch.zeros(1, dtype=torch.int32, device=dev)
        pattern = (sp[0] != 0xFF).astype(np.uint8)
        dls_count_async_ex(n, kflags, pattern, d_pre, len(sel), d_cnt, d_st, stream, lc)
        torch.cuda.synchronize()
        ms, _ = dls_kernel_time_ms(stream)
        if int(d_st.item()):
            raise RuntimeError(f"device status {int(d_st.item())} in batch {b}")
        c = d_cnt.cpu().numpy().view(np.uint64)
        m = mult[sel]
        ws = int((c.astype(object) * m.astype(object)).sum())
        state["weighted_sum"] = str(int(state["weighted_sum"]) + ws)
        state["squares"] = str(int(state["squares"]) + int(c.astype(object).sum()))
        state["kernel_seconds"] += ms * 1e-3
        state["done_batches"] = b + 1
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(state, f)
        os.replace(tmp, path)
        log(f"batch {b + 1}/{batches}: {len(sel)} workunits, {ms * 1e-3:.1f} s, "
            f"{int(c.astype(object).sum()) / (ms * 1e-3):.3e} squares/s")
        del d_pre, d_cnt
    return state


def merge(out: str) -> dict:
    files = sorted(glob.glob(os.path.join(out, "chunk_*_of_*.json")))
    if not files:
        raise RuntimeError(f"no chunk files in {out}")
    parts = []
    for p in files:
        with open(p) as f:
            parts.append(json.load(f))
    first = parts[0]
    keys = ("n", "flags", "depth", "chunks", "workunits", "split_digest")
    for q in parts:
        if any(q[k] != first[k] for k in keys):
            raise RuntimeError("chunk files come from different splits")
    chunks = first["chunks"]
    have = {q["chunk"] for q in parts if q["done_batches"] == q["batches"]}
    missing = sorted(set(range(chunks)) - have)
    total = sum(int(q["weighted_sum"]) for q in parts)
    return {"n": first["n"], "flags": first["flags"], "depth": first["depth"], "chunks": chunks,
            "complete": not missing, "missing_chunks": missing, "weighted_sum": total,
            "squares": sum(int(q["squares"]) for q in parts),
            "kernel_seconds": sum(q["kernel_seconds"] for q in parts)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=9)
    ap.add_argument("--symbreak", action="store_true")
    ap.add_argument("--vsym", action="store_true")
    ap.add_argument("--depth", type=int, default=22)
    ap.add_argument("--chunks", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--batches", type=int, default=10)
    ap.add_argument("--launch", default="{}", help="launch settings as JSON, e.g. '{\"order_variant\": 2}'; "
                    "empty: the autotuner's order9-sample entry for order 9 with --symbreak")
    ap.add_argument("--out", default="fullcount_out")
    ap.add_argument("--split-cache", default=None, help="file holding the split, shared by the chunks")
    ap.add_argument("--merge", default=None, help="sum the chunk files of this directory")
    args = ap.parse_args(argv)
    if args.merge:
        print(json.dumps(merge(args.merge)), flush=True)
        return
    flags = (DLS_SYMBREAK if args.symbreak else 0) | (DLS_VSYM if args.vsym else 0)
    launch = json.loads(args.launch)
    if not launch and args.n == 9 and flags == DLS_SYMBREAK:
        # the autotuner's launch for a sample of this workload, if tuned here
        from . import autotune
        tuned = autotune.best(9, 0, "order9-sample")
        launch = {k: v for k, v in (tuned or {}).items() if k != "ms"}
    print(f"launch: {launch or 'library defaults'}", flush=True)
    st = run_chunk(args.n, flags, args.depth, args.chunk, args.chunks, args.out, args.batches,
                   launch, log=lambda s: print(s, flush=True), split_cache=args.split_cache)
    print(json.dumps(st), flush=True)


if __name__ == "__main__":
    sys.exit(main())
