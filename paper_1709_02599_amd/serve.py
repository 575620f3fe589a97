"""Serving loop: counting requests that arrive over time, batched continuously
on one GPU by the library's serving kernel.

A request is (order N, flags, prefix); its answer is the exact number of DLS
(VS-DLS with DLS_VSYM) that agree with the prefix.  The loop holds one
library server (`dls_server_create`): a long-running kernel on its own
stream that serves every order 4..9 with or without vertical symmetry, a
ring of job slots and a pool of workunit cells in host-pinned memory.  The
loop

* admits waiting requests in arrival order as long as the server accepts
  them: the server splits the prefix into workunits (Sec. 5.2), writes them
  to the pool and publishes the job in its ring, or answers "no room"
  (DLS_EBUSY) when no ring slot or no pool room is free -- admission follows
  the library's real allocation;
* never launches anything per request: the running kernel takes published
  jobs as their waves free up, so requests admitted while others run are
  counted on the device at the same time, and the kernel computes each
  request's total;
* retires a request when the server reports it done (a completion record the
  kernel writes to host-pinned memory) and frees its slot and pool room.

Latencies are measured from a request's arrival to its retirement.  Every
count comes from the GPU kernels; nothing here computes one.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import (DLS_VSYM, dls_server_create, dls_server_destroy, dls_server_info, dls_server_poll,
               dls_server_shared, dls_server_submit)

EMPTY = 0xFF
TICK_S = 1e-8          # s_memrealtime runs at 100 MHz


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
    n: int = 0
    vs: bool = False
    dev_start: int = 0            # device ticks: first chunk taken
    dev_end: int = 0              # device ticks: last piece finished

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Continuous batching of requests over the library's serving kernel."""

    def __init__(self, pool_bytes: int = 256 << 20, max_jobs: int = 128, min_tasks: int = 16384,
                 launch: Optional[dict] = None):
        self.pool_bytes = pool_bytes
        self.min_tasks = min_tasks
        self.handle = dls_server_create(max_jobs, pool_bytes, launch)
        self.peak_pool_used = 0
        self.busy_answers = 0         # admissions the server refused for lack of room
        self.peak_in_flight = 0

    def info(self) -> dict:
        return dls_server_info(self.handle)

    def shared(self) -> int:
        """Subtrees handed between waves so far (requests retired)."""
        return dls_server_shared(self.handle)

    def close(self) -> None:
        if self.handle:
            dls_server_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, requests: List[Request], realtime: bool = True, timeout: float = 120.0) -> List[Result]:
        """Serve `requests` (released at their arrival times with realtime,
        else all at once); returns results ordered by request id."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        running: Dict[int, tuple] = {}     # ticket -> (request, admitted)
        results: List[Result] = []
        h = self.handle
        t0 = time.perf_counter()
        while pending or waiting or running:
            now = time.perf_counter() - t0
            if now > timeout:
                raise TimeoutError(f"{len(running)} requests still running after {timeout} s")
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # admit in arrival order while the server has room
            while waiting:
                req = waiting[0]
                ticket = dls_server_submit(h, req.n, DLS_VSYM if req.vs else 0, req.prefix, self.min_tasks)
                if ticket is None:
                    self.busy_answers += 1
                    break
                waiting.popleft()
                running[ticket] = (req, time.perf_counter() - t0)
            self.peak_in_flight = max(self.peak_in_flight, len(running))
            self.peak_pool_used = max(self.peak_pool_used, self.pool_bytes - dls_server_info(h)["pool_free"])
            # retire finished requests
            for ticket, (req, adm) in list(running.items()):
                done, count, ticks = dls_server_poll(h, ticket)
                if done:
                    results.append(Result(req.rid, count, req.arrival if realtime else 0.0, adm,
                                          time.perf_counter() - t0, req.n, req.vs, ticks[0], ticks[1]))
                    del running[ticket]
            if pending and realtime and not waiting and not running:
                time.sleep(max(0.0, min(0.002, pending[0].arrival - (time.perf_counter() - t0))))
            elif running or waiting:
                time.sleep(0.00005)
        return sorted(results, key=lambda r: r.rid)


def overlapping_pairs(results: List[Result]) -> int:
    """Number of pairs of requests whose device intervals (first chunk taken,
    last piece finished) overlap: requests counted on the GPU at the same
    time.  Requests that needed no device work are left out."""
    iv = sorted((r.dev_start, r.dev_end) for r in results if r.dev_end > 0)
    pairs = 0
    ends: List[int] = []
    for s, e in iv:
        ends = [x for x in ends if x > s]
        pairs += len(ends)
        ends.append(e)
    return pairs


def max_concurrency(results: List[Result]) -> int:
    """Largest number of requests in progress on the device at one moment."""
    ev = []
    for r in results:
        if r.dev_end > 0:
            ev.append((r.dev_start, 1))
            ev.append((r.dev_end, -1))
    ev.sort(key=lambda x: (x[0], x[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


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


def sweep(jobs: int = 200, fractions=(0.25, 0.5, 0.75, 0.9, 1.1), seed: Optional[int] = None,
          server: Optional[Server] = None, emit=print) -> List[dict]:
    """Closed-loop capacity first (all requests waiting), then Poisson
    arrivals at fractions of it; one dict per rate."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import dls_workloads
    seed = dls_workloads.DEFAULT_SEED if seed is None else seed

    def requests(rate, s):
        return [Request(j.jid, j.n, j.vs, j.prefix, j.arrival) for j in dls_workloads.job_stream(jobs, rate, seed=s)]

    own = server is None
    srv = server or Server()
    rows = []
    try:
        srv.run(requests(1.0, seed + 1)[:16], realtime=False)          # warm-up
        reqs = requests(1.0, seed)
        sh = srv.shared()
        t = time.perf_counter()
        res = srv.run(reqs, realtime=False)
        wall = time.perf_counter() - t
        cap = len(res) / wall
        row = {"mode": "closed-loop", "jobs": len(res), "seconds": wall, "jobs_per_s": cap,
               "squares_per_s": sum(r.count for r in res) / wall, "max_concurrency": max_concurrency(res),
               "subtrees_shared": srv.shared() - sh, **latency_stats(res)}
        rows.append(row)
        emit(row)
        for frac in fractions:
            rate = frac * cap
            reqs = requests(rate, seed)
            sh = srv.shared()
            t = time.perf_counter()
            res = srv.run(reqs, realtime=True)
            wall = time.perf_counter() - t
            row = {"mode": "poisson", "load": frac, "rate_jobs_per_s": rate, "jobs": len(res), "seconds": wall,
                   "jobs_per_s": len(res) / wall, "squares_per_s": sum(r.count for r in res) / wall,
                   "max_concurrency": max_concurrency(res), "subtrees_shared": srv.shared() - sh,
                   **latency_stats(res)}
            rows.append(row)
            emit(row)
    finally:
        if own:
            srv.close()
    return rows


def solo_times(jobs: int = 200, min_tasks: int = 16384, seed: Optional[int] = None) -> dict:
    """Each request of the stream counted alone by the batch path (its
    workunits from dls_split_target, one dls_count_async_ex launch timed with
    the library's kernel events): the search work the mix holds, to compare
    with the serving kernel's latencies."""
    import os
    import sys
    import torch
    from . import DlsLaunch, dls_count_async_ex, dls_kernel_time_ms, dls_split_target
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import dls_workloads
    seed = dls_workloads.DEFAULT_SEED if seed is None else seed
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = []
    for j in dls_workloads.job_stream(jobs, 1.0, seed=seed):
        flags = DLS_VSYM if j.vs else 0
        units = dls_split_target(j.n, flags, j.prefix, min_tasks, 24)
        if len(units) == 0:
            continue
        pattern = (units[0] != EMPTY).astype(np.uint8)
        d_pre = torch.from_numpy(np.ascontiguousarray(units)).to(dev)
        d_cnt = torch.zeros(len(units), dtype=torch.int64, device=dev)
        d_st = torch.zeros(1, dtype=torch.int32, device=dev)
        dls_count_async_ex(j.n, flags, pattern, d_pre, len(units), d_cnt, d_st, stream, DlsLaunch(time_kernel=1))
        torch.cuda.synchronize()
        ms, _ = dls_kernel_time_ms(stream)
        rows.append({"rid": j.jid, "n": j.n, "vs": bool(j.vs), "workunits": len(units), "kernel_ms": ms,
                     "count": int(d_cnt.sum().item())})
    rows.sort(key=lambda r: -r["kernel_ms"])
    return {"requests_searched": len(rows), "total_kernel_ms": sum(r["kernel_ms"] for r in rows),
            "largest": rows[:5]}


def main(argv=None):
    """Rate sweep; prints one JSON line per rate."""
    import argparse
    import json

    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=200)
    ap.add_argument("--fractions", default="0.25,0.5,0.75,0.9,1.1")
    ap.add_argument("--min-tasks", type=int, default=16384)
    ap.add_argument("--blocks-per-cu", type=int, default=1)
    ap.add_argument("--steal-depth", type=int, default=0,
                    help="handing of subtrees between waves: 0 = library default, < 0 = off")
    ap.add_argument("--solo", action="store_true",
                    help="instead of the sweep: each request counted alone by the batch path")
    args = ap.parse_args(argv)
    if args.solo:
        print(json.dumps(solo_times(args.jobs, args.min_tasks)), flush=True)
        return
    with Server(min_tasks=args.min_tasks,
                launch={"blocks_per_cu": args.blocks_per_cu, "steal_depth": args.steal_depth}) as srv:
        sweep(args.jobs, [float(x) for x in args.fractions.split(",")], server=srv,
              emit=lambda row: print(json.dumps(row), flush=True))


if __name__ == "__main__":
    main()
