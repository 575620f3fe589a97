"""Serving loop: counting requests that arrive over time, batched continuously
onto one GPU.

A request is (order N, flags, prefix); its answer is the exact number of DLS
(VS-DLS with DLS_VSYM) that agree with the prefix.  The loop

* admits a waiting request as soon as one of `slots` execution slots is free
  and its device memory fits the budget (`mem_budget` bytes of prefixes,
  task records and counts in flight);
* launches the request's prefix on the slot's own HIP stream: the library
  deepens it on the device (breadth-first passes, the split of Sec. 5.2 done
  on the GPU) into enough tasks for the slot's share of the chip, then runs
  the persistent kernel; requests admitted while others run execute on the
  device at the same time; the per-request total is reduced on the device.
  (With host_split, the prefix is instead split on the host into at least
  min_tasks workunits before the launch.)
* retires a request when its stream's event completes and frees its slot and
  memory for the next one.

Latencies are measured from a request's arrival to its retirement.  Every
count comes from the GPU kernels; nothing here computes one.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import (DLS_VSYM, DlsLaunch, dls_count_async_ex, dls_split_from, _lib)

EMPTY = 0xFF


@dataclass
class Request:
    rid: int
    n: int
    vs: bool
    prefix: np.ndarray
    arrival: float = 0.0          # seconds after the stream start


@dataclass
class Result:
    rid: int
    count: int
    arrival: float
    admitted: float
    done: float
    tasks: int
    n: int = 0
    vs: bool = False

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _split_target(n: int, flags: int, prefix: np.ndarray, target: int, max_depth: int = 12):
    """Shallowest split of `prefix` with at least `target` workunits (or the
    deepest tried).  Returns the workunits [P, n*n]."""
    num = ctypes.c_int64(0)
    best = 0
    for depth in range(0, max_depth + 1):
        rc = _lib.dls_split_from(n, flags, prefix.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                 depth, None, 0, ctypes.byref(num))
        if rc != 0:
            break
        best = depth
        if num.value >= target or num.value == 0:
            break
    return dls_split_from(n, flags, prefix, best)


class Server:
    def __init__(self, slots: int = 4, mem_budget: int = 1 << 30, min_tasks: int = 4096,
                 device: int = 0, host_split: bool = False, expand_target: int = 1 << 15):
        import torch
        self.torch = torch
        self.dev = torch.device(f"cuda:{device}")
        self.slots = slots
        self.mem_budget = mem_budget
        self.min_tasks = min_tasks
        self.host_split = host_split
        self.expand_target = expand_target
        # default-priority streams, one per execution slot
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(slots)]
        self.free = list(range(slots))
        self.mem_used = 0
        self.cus = torch.cuda.get_device_properties(self.dev).multi_processor_count

    def _bytes(self, n: int, tasks: int) -> int:
        return tasks * (n * n + 80 + 8) + 4096

    def _launch(self, slot: int, req: Request, tasks: np.ndarray):
        torch = self.torch
        st = self.streams[slot]
        flags = DLS_VSYM if req.vs else 0
        with torch.cuda.stream(st):
            d_pre = torch.from_numpy(tasks).to(self.dev, non_blocking=False)
            d_cnt = torch.empty(max(1, len(tasks)), dtype=torch.int64, device=self.dev)
            d_st = torch.zeros(1, dtype=torch.int32, device=self.dev)
        if self.host_split:
            # grid sized to the batch: one resident workgroup per CU for small
            # batches so that several requests share the chip, more for big ones
            bpc = int(min(8, max(1, len(tasks) // (self.cus * 256))))
            launch = DlsLaunch(block=256, blocks_per_cu=bpc, steal_depth=0, refill_every=0, expand_target=-1)
        else:
            # each slot gets an equal share of the chip's resident workgroups
            bpc = max(1, 8 // self.slots)
            launch = DlsLaunch(block=256, blocks_per_cu=bpc, expand_target=self.expand_target)
        pattern = (tasks[0] != EMPTY).astype(np.uint8)
        dls_count_async_ex(req.n, flags, pattern, d_pre, len(tasks), d_cnt, d_st, st, launch)
        with torch.cuda.stream(st):
            total = d_cnt[:len(tasks)].sum()
            ev = torch.cuda.Event()
            ev.record(st)
        return {"pre": d_pre, "cnt": d_cnt, "st": d_st, "total": total, "event": ev}

    def run(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Serve `requests` (sorted by arrival).  With realtime, requests are
        released at their arrival times; otherwise all are available at once."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        running: Dict[int, tuple] = {}
        results: List[Result] = []
        t0 = time.perf_counter()
        while pending or waiting or running:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # retire finished requests
            for slot, (req, job, adm, nbytes, ntask) in list(running.items()):
                if job["event"].query():
                    status = int(job["st"].item())
                    if status:
                        raise RuntimeError(f"request {req.rid}: device status {status}")
                    count = int(job["total"].item()) if ntask else 0
                    results.append(Result(req.rid, count, req.arrival if realtime else 0.0, adm,
                                          time.perf_counter() - t0, ntask, req.n, req.vs))
                    self.mem_used -= nbytes
                    self.free.append(slot)
                    del running[slot]
            # admit while a slot and memory are free
            while waiting and self.free:
                req = waiting[0]
                flags = DLS_VSYM if req.vs else 0
                if self.host_split:
                    tasks = _split_target(req.n, flags, req.prefix, self.min_tasks)
                else:
                    tasks = np.ascontiguousarray(req.prefix.reshape(1, -1), dtype=np.uint8)
                nbytes = self._bytes(req.n, len(tasks))
                if running and self.mem_used + nbytes > self.mem_budget:
                    break
                waiting.popleft()
                slot = self.free.pop()
                adm = time.perf_counter() - t0
                if len(tasks) == 0:
                    results.append(Result(req.rid, 0, req.arrival if realtime else 0.0, adm, adm, 0,
                                          req.n, req.vs))
                    self.free.append(slot)
                    continue
                job = self._launch(slot, req, tasks)
                self.mem_used += nbytes
                running[slot] = (req, job, adm, nbytes, len(tasks))
            if running or waiting:
                time.sleep(0.0002)
            elif pending and realtime:
                time.sleep(max(0.0, min(0.002, pending[0].arrival - (time.perf_counter() - t0))))
        torch.cuda.synchronize()
        return sorted(results, key=lambda r: r.rid)


def _stats(lat) -> dict:
    lat = np.asarray(lat)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "n": int(len(lat))}


def latency_stats(results: List[Result]) -> dict:
    """p50/p99/mean latency overall and per order N."""
    out = _stats([r.latency for r in results])
    per = {}
    for n in sorted({r.n for r in results}):
        per[str(n)] = _stats([r.latency for r in results if r.n == n])
    out["per_order"] = per
    return out


def main(argv=None):
    """Rate sweep: closed-loop capacity first (all requests waiting), then
    Poisson arrivals at fractions of it.  Prints one JSON line per rate."""
    import argparse
    import json
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import dls_workloads

    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--fractions", default="0.25,0.5,0.75,0.9,1.1")
    ap.add_argument("--seed", type=int, default=dls_workloads.DEFAULT_SEED)
    ap.add_argument("--host-split", action="store_true")
    ap.add_argument("--expand-target", type=int, default=1 << 15)
    args = ap.parse_args(argv)

    def requests(rate, seed):
        jobs = dls_workloads.job_stream(args.jobs, rate, seed=seed)
        return [Request(j.jid, j.n, j.vs, j.prefix, j.arrival) for j in jobs]

    srv = Server(slots=args.slots, host_split=args.host_split, expand_target=args.expand_target)
    warm = requests(1.0, args.seed + 1)[:8]
    srv.run(warm, realtime=False)
    reqs = requests(1.0, args.seed)
    t = time.perf_counter()
    res = srv.run(reqs, realtime=False)
    wall = time.perf_counter() - t
    cap = len(res) / wall
    squares = sum(r.count for r in res)
    print(json.dumps({"mode": "closed-loop", "jobs": len(res), "seconds": wall, "jobs_per_s": cap,
                      "squares_per_s": squares / wall, **latency_stats(res)}), flush=True)
    for frac in [float(x) for x in args.fractions.split(",")]:
        rate = frac * cap
        reqs = requests(rate, args.seed)
        t = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        wall = time.perf_counter() - t
        squares = sum(r.count for r in res)
        print(json.dumps({"mode": "poisson", "load": frac, "rate_jobs_per_s": rate, "jobs": len(res),
                          "seconds": wall, "squares_per_s": squares / wall, **latency_stats(res)}),
              flush=True)


if __name__ == "__main__":
    main()
