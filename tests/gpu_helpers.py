"""Helpers for GPU tests: run the library's kernels through the C ABI on
torch device buffers."""
import numpy as np

EMPTY = 0xFF


def gpu_counts(dls, n, flags, prefixes, plain=False, launch=None, stream=None, steps=False):
    """Per-prefix counts from dls_count_async_ex (all prefixes share the
    first prefix's assigned cells).  Returns (counts uint64, status[, steps])."""
    import torch
    pre = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint8).reshape(-1, n * n))
    num = pre.shape[0]
    dev = torch.device("cuda:0")
    d_pre = torch.from_numpy(pre).to(dev)
    d_cnt = torch.zeros(max(1, num), dtype=torch.int64, device=dev)
    d_status = torch.zeros(1, dtype=torch.int32, device=dev)
    d_steps = torch.zeros(2, dtype=torch.int64, device=dev)
    pattern = (pre[0] != EMPTY).astype(np.uint8) if num else None
    fl = flags | (dls.DLS_PLAIN if plain else 0)
    st = stream if stream is not None else torch.cuda.current_stream()
    if steps:
        dls.dls_count_async_stats(n, fl, pattern, d_pre, num, d_cnt, d_status, st, launch, d_steps)
    else:
        dls.dls_count_async_ex(n, fl, pattern, d_pre, num, d_cnt, d_status, st, launch)
    torch.cuda.synchronize()
    counts = d_cnt.cpu().numpy().view(np.uint64)[:num].copy()
    status = int(d_status.item())
    if steps:
        return counts, status, int(d_steps[0].item())
    return counts, status


def weighted_total(counts, mult):
    return int((np.asarray(counts).astype(object) * np.asarray(mult).astype(object)).sum())
