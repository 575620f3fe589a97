"""One counting step -- task preparation, the search kernel and the weighted
reduction of the counts -- captured into a HIP graph and replayed.

The library allocates its per-stream scratch on the first call on a stream
and when a batch is larger than any before on it; neither may happen under
capture (the call then returns DLS_ECAPTURE), so a `CountStep` makes one
uncaptured call on its own stream before it captures.  The captured work
holds no memset: the queue control block, the donation flags and the
reduction's output are cleared by kernels, so every replay starts from the
same state and recomputes every count.

Replays of one step must not overlap each other or eager calls on the step's
stream (they share its scratch): `replay()` issues on that stream.
"""
from __future__ import annotations

from typing import Optional

from . import DlsLaunch, dls_count_async_ex, dls_reduce_weighted


class CountStep:
    def __init__(self, n: int, flags: int, pattern, d_prefixes, num: int, d_counts, d_status,
                 d_mult=None, launch: Optional[DlsLaunch] = None, device=None):
        import torch
        self.torch = torch
        self.args = (n, flags, pattern, d_prefixes, num, d_counts, d_status)
        self.d_mult = d_mult
        self.launch = launch
        dev = device if device is not None else d_counts.device
        self.stream = torch.cuda.Stream(device=dev)   # default priority
        self.total = torch.zeros(1, dtype=torch.int64, device=dev)
        self.graph = None

    def _issue(self):
        n, flags, pattern, d_pre, num, d_cnt, d_st = self.args
        dls_count_async_ex(n, flags, pattern, d_pre, num, d_cnt, d_st, self.stream, self.launch)
        dls_reduce_weighted(d_cnt, self.d_mult, num, self.total, self.stream)

    def eager(self):
        """Issue the step without a graph (on the step's stream)."""
        self._issue()
        return self.total

    def capture(self):
        torch = self.torch
        # the uncaptured call sizes this stream's scratch for the batch
        self._issue()
        self.stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self._issue()
        self.graph = g
        return self

    def replay(self):
        if self.graph is None:
            raise RuntimeError("CountStep.capture() has not run")
        with self.torch.cuda.stream(self.stream):
            self.graph.replay()
        return self.total
