"""Python binding of libdls.so (include/dls.h): exact counting of diagonal
Latin squares on MI355X (gfx950).

The functions below carry the C ABI's names and only marshal arguments:
NumPy arrays for host buffers, torch tensors (``.data_ptr()``) for device
buffers and ``torch.cuda.Stream`` (or a raw handle) for streams.  Every step
of the count runs in the HIP library; there is no Python or CPU fallback.
If the library has not been built, importing this package raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "DLS_VSYM", "DLS_SYMBREAK", "DLS_PLAIN", "DLS_EMPTY", "DLSError", "LIB_PATH",
    "dls_version", "dls_strerror", "dls_last_hip_error", "dls_order", "dls_split", "dls_split_from",
    "dls_split_sample", "dls_group_order", "dls_canon", "dls_count", "dls_count_async", "dls_stream_status",
    "dls_count_async_ex", "dls_count_async_noalloc", "dls_count_async_stats", "dls_valu_probe", "DlsLaunch",
    "dls_order_variant", "dls_reduce_weighted", "dls_kernel_time_ms", "dls_count_cells",
    "dls_count_cells_async", "dls_split_cells", "dls_order_cost",
    "dls_hourglass_classes_async", "hourglass_classes_gpu", "DLS_EBUSY", "dls_server_create",
    "dls_server_submit", "dls_server_poll", "dls_server_info", "dls_server_waves", "dls_server_shared", "dls_server_destroy",
    "dls_split_target",
]

DLS_VSYM = 1 << 0
DLS_SYMBREAK = 1 << 1
DLS_PLAIN = 1 << 2
DLS_EMPTY = 0xFF
DLS_ECAPTURE = -6
DLS_EBUSY = -7

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdls.so")


class DLSError(RuntimeError):
    def __init__(self, code: int, what: str):
        detail = _lib.dls_last_hip_error().decode() if code == -4 else ""
        super().__init__(f"{what}: {dls_strerror(code)} ({code}) {detail}".rstrip())
        self.code = code


class DlsLaunch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("steal_depth", ctypes.c_int), ("refill_every", ctypes.c_int),
                ("order_variant", ctypes.c_int), ("time_kernel", ctypes.c_int),
                ("expand_target", ctypes.c_int), ("chunk_min", ctypes.c_int), ("lds_masks", ctypes.c_int),
                ("refill_min", ctypes.c_int), ("wg_pool", ctypes.c_int)]


def _load() -> ctypes.CDLL:
    # torch ships its own HIP runtime under the same soname as the system's.
    # Loading torch first makes libdls.so bind to that already-loaded runtime;
    # the other order would put two HIP runtimes in one process, and device
    # pointers from torch would be foreign to the library's runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950) before using paper_1709_02599_amd")
    lib = ctypes.CDLL(LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    sig = {
        "dls_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "dls_version": (ctypes.c_char_p, []),
        "dls_last_hip_error": (ctypes.c_char_p, []),
        "dls_order": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, u8p,
                                     ctypes.POINTER(ctypes.c_int)]),
        "dls_split": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, u8p, u32p,
                                     ctypes.c_int64, i64p]),
        "dls_split_from": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, ctypes.c_int, u8p,
                                          ctypes.c_int64, i64p]),
        "dls_split_sample": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.c_int, i64p,
                                            ctypes.c_int64, u8p, i64p]),
        "dls_group_order": (ctypes.c_int64, [ctypes.c_int]),
        "dls_canon": (ctypes.c_int, [ctypes.c_int, u8p, u32p]),
        "dls_count": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_uint64)]),
        "dls_count_async": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, vp, ctypes.c_int64, vp, vp]),
        "dls_stream_status": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint32)]),
        "dls_count_async_ex": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, vp,
                                              ctypes.c_int64, vp, vp, vp,
                                              ctypes.POINTER(DlsLaunch)]),
        "dls_count_async_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, vp,
                                                   ctypes.c_int64, vp, vp, vp,
                                                   ctypes.POINTER(DlsLaunch)]),
        "dls_count_async_stats": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, vp,
                                                 ctypes.c_int64, vp, vp, vp,
                                                 ctypes.POINTER(DlsLaunch), vp]),
        "dls_valu_probe": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, vp]),
        "dls_order_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, ctypes.c_int, u8p,
                                             ctypes.POINTER(ctypes.c_int)]),
        "dls_reduce_weighted": (ctypes.c_int, [vp, vp, ctypes.c_int64, vp, vp]),
        "dls_kernel_time_ms": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_int64)]),
        "dls_split_cells": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, ctypes.POINTER(ctypes.c_int),
                                           ctypes.c_int, u8p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
        "dls_order_cost": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                          u8p, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64),
                                          ctypes.POINTER(ctypes.c_uint64)]),
        "dls_hourglass_classes_async": (ctypes.c_int, [ctypes.c_int, vp, ctypes.c_int64, vp, vp, ctypes.c_int64,
                                                       vp, vp, vp]),
        "dls_count_cells": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int),
                                           ctypes.c_int, u8p, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]),
        "dls_count_cells_async": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int),
                                                 ctypes.c_int, u8p, vp, ctypes.c_int64, vp, vp, vp,
                                                 ctypes.POINTER(DlsLaunch)]),
    }
    sig.update({
        "dls_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(DlsLaunch),
                                             ctypes.POINTER(vp)]),
        "dls_server_submit": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_uint32, u8p, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64)]),
        "dls_server_poll": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64),
                                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int)]),
        "dls_server_info": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]),
        "dls_server_waves": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "dls_server_shared": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64)]),
        "dls_server_destroy": (ctypes.c_int, [vp]),
        "dls_split_target": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint32, u8p, ctypes.c_int64, ctypes.c_int, u8p,
                                            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    })
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise DLSError(rc, what)


def _square(n: int, cells) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(cells, dtype=np.uint8).reshape(n * n))


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or an int), None for None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(s) -> Optional[int]:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def dls_strerror(code: int) -> str:
    return _lib.dls_strerror(code).decode()


def dls_version() -> str:
    return _lib.dls_version().decode()


def dls_last_hip_error() -> str:
    return _lib.dls_last_hip_error().decode()


def dls_order(n: int, flags: int = 0, assigned=None) -> list:
    """Fill order of the empty cells (flat indices).  ``assigned`` defaults to
    row 0."""
    if assigned is None:
        assigned = np.zeros(n * n, dtype=np.uint8)
        assigned[:n] = 1
    a = _square(n, assigned)
    out = np.zeros(max(1, n * n), dtype=np.uint8)
    ln = ctypes.c_int(0)
    _check(_lib.dls_order(n, flags, _u8(a), _u8(out), ctypes.byref(ln)), "dls_order")
    return [int(x) for x in out[:ln.value]]


def dls_split(n: int, flags: int, depth: int) -> Tuple[np.ndarray, np.ndarray]:
    """Workunit prefixes [P, n*n] uint8 and class powers [P] uint32."""
    num = ctypes.c_int64(0)
    _check(_lib.dls_split(n, flags, depth, None, None, 0, ctypes.byref(num)), "dls_split")
    p = num.value
    pre = np.zeros((p, n * n), dtype=np.uint8)
    mult = np.zeros(p, dtype=np.uint32)
    if p:
        _check(_lib.dls_split(n, flags, depth, _u8(pre),
                              mult.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), p,
                              ctypes.byref(num)), "dls_split")
    return pre, mult


def dls_split_from(n: int, flags: int, base, depth: int) -> np.ndarray:
    b = _square(n, base)
    num = ctypes.c_int64(0)
    _check(_lib.dls_split_from(n, flags, _u8(b), depth, None, 0, ctypes.byref(num)),
           "dls_split_from")
    p = num.value
    pre = np.zeros((p, n * n), dtype=np.uint8)
    if p:
        _check(_lib.dls_split_from(n, flags, _u8(b), depth, _u8(pre), p, ctypes.byref(num)),
               "dls_split_from")
    return pre


def dls_split_sample(n: int, flags: int, depth: int,
                     indices: Sequence[int]) -> Tuple[np.ndarray, int]:
    idx = np.ascontiguousarray(np.asarray(indices, dtype=np.int64))
    out = np.zeros((len(idx), n * n), dtype=np.uint8)
    tot = ctypes.c_int64(0)
    _check(_lib.dls_split_sample(n, flags, depth,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(idx),
                                 _u8(out), ctypes.byref(tot)), "dls_split_sample")
    return out, int(tot.value)


def dls_group_order(n: int) -> int:
    r = _lib.dls_group_order(n)
    if r < 0:
        raise DLSError(int(r), "dls_group_order")
    return int(r)


def dls_canon(n: int, h) -> int:
    m = ctypes.c_uint32(0)
    _check(_lib.dls_canon(n, _u8(_square(n, h)), ctypes.byref(m)), "dls_canon")
    return int(m.value)


def dls_count(n: int, flags: int, prefixes) -> np.ndarray:
    """Exact per-prefix counts on the GPU (host buffers, blocking)."""
    p = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint8).reshape(-1, n * n))
    out = np.zeros(p.shape[0], dtype=np.uint64)
    if p.shape[0]:
        _check(_lib.dls_count(n, flags, _u8(p), p.shape[0],
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "dls_count")
    return out


def _pattern(n: int, pattern) -> Optional[np.ndarray]:
    if pattern is None:
        return None
    return _square(n, np.asarray(pattern).astype(bool).astype(np.uint8))


def _launch(launch) -> Optional[DlsLaunch]:
    if launch is None:
        return None
    if isinstance(launch, DlsLaunch):
        return launch
    return DlsLaunch(**launch)


def dls_count_async(n: int, flags: int, d_prefixes, num: int, d_counts, stream=None) -> None:
    """Counts of device prefixes into device counts on `stream`; the pattern
    of assigned cells is read from prefix 0."""
    _check(_lib.dls_count_async(n, flags, _ptr(d_prefixes), num, _ptr(d_counts), _stream(stream)),
           "dls_count_async")


def dls_stream_status(stream=None) -> int:
    """Status bits of the calls made on `stream` without a status buffer
    (waits for the stream; clears them)."""
    v = ctypes.c_uint32(0)
    _check(_lib.dls_stream_status(_stream(stream), ctypes.byref(v)), "dls_stream_status")
    return int(v.value)


def dls_count_async_ex(n: int, flags: int, pattern, d_prefixes, num: int, d_counts,
                       d_status=None, stream=None, launch=None) -> None:
    pat = _pattern(n, pattern)
    lc = _launch(launch)
    _check(_lib.dls_count_async_ex(n, flags, None if pat is None else _u8(pat), _ptr(d_prefixes),
                                   num, _ptr(d_counts), _ptr(d_status), _stream(stream),
                                   None if lc is None else ctypes.byref(lc)),
           "dls_count_async_ex")


def dls_count_async_noalloc(n: int, flags: int, pattern, d_prefixes, num: int, d_counts,
                            d_status, stream=None, launch=None) -> None:
    """dls_count_async_ex without any device allocation (scratch in the
    library's static device array; overlapping calls on one GPU race)."""
    pat = _pattern(n, pattern)
    lc = _launch(launch)
    _check(_lib.dls_count_async_noalloc(n, flags, None if pat is None else _u8(pat), _ptr(d_prefixes),
                                        num, _ptr(d_counts), _ptr(d_status), _stream(stream),
                                        None if lc is None else ctypes.byref(lc)),
           "dls_count_async_noalloc")


def dls_count_async_stats(n: int, flags: int, pattern, d_prefixes, num: int, d_counts,
                          d_status=None, stream=None, launch=None, d_steps=None) -> None:
    pat = _pattern(n, pattern)
    lc = _launch(launch)
    _check(_lib.dls_count_async_stats(n, flags, None if pat is None else _u8(pat),
                                      _ptr(d_prefixes), num, _ptr(d_counts), _ptr(d_status),
                                      _stream(stream), None if lc is None else ctypes.byref(lc),
                                      _ptr(d_steps)), "dls_count_async_stats")


def dls_valu_probe(blocks: int, iters: int, d_sink, stream=None) -> None:
    _check(_lib.dls_valu_probe(blocks, iters, _ptr(d_sink), _stream(stream)), "dls_valu_probe")


def dls_order_variant(n: int, flags: int, assigned, variant: int) -> list:
    a = _square(n, assigned)
    out = np.zeros(max(1, n * n), dtype=np.uint8)
    ln = ctypes.c_int(0)
    _check(_lib.dls_order_variant(n, flags, _u8(a), variant, _u8(out), ctypes.byref(ln)),
           "dls_order_variant")
    return [int(x) for x in out[:ln.value]]


def dls_reduce_weighted(d_counts, d_mult, num: int, d_out, stream=None) -> None:
    _check(_lib.dls_reduce_weighted(_ptr(d_counts), _ptr(d_mult), num, _ptr(d_out),
                                    _stream(stream)), "dls_reduce_weighted")


def dls_kernel_time_ms(stream=None):
    """(mean ms, launches) of the search kernels timed on `stream` since the
    previous call; the stream must have been synchronised."""
    ms = ctypes.c_float(0.0)
    k = ctypes.c_int64(0)
    _check(_lib.dls_kernel_time_ms(_stream(stream), ctypes.byref(ms), ctypes.byref(k)),
           "dls_kernel_time_ms")
    return float(ms.value), int(k.value)


def _cells(cells):
    arr = np.ascontiguousarray(np.asarray(list(cells), dtype=np.int32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(arr)


def dls_count_cells(n: int, flags: int, cells, prefixes) -> np.ndarray:
    """Partial squares: for each prefix, the number of consistent assignments
    of exactly `cells` (Sec. 5.3's incomplete squares)."""
    keep, cp, nc = _cells(cells)
    pre = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint8).reshape(-1, n * n))
    out = np.zeros(len(pre), dtype=np.uint64)
    _check(_lib.dls_count_cells(n, flags, cp, nc, _u8(pre), len(pre),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), "dls_count_cells")
    del keep
    return out


def dls_count_cells_async(n: int, flags: int, cells, pattern, d_prefixes, num: int, d_counts,
                          d_status=None, stream=None, launch=None) -> None:
    keep, cp, nc = _cells(cells)
    pat = _pattern(n, pattern)
    lc = _launch(launch)
    _check(_lib.dls_count_cells_async(n, flags, cp, nc, None if pat is None else _u8(pat), _ptr(d_prefixes),
                                      num, _ptr(d_counts), _ptr(d_status), _stream(stream),
                                      None if lc is None else ctypes.byref(lc)), "dls_count_cells_async")
    del keep


def dls_split_cells(n: int, flags: int, base, cells) -> np.ndarray:
    """Every consistent assignment of exactly `cells` on top of `base`
    ([P, n*n] uint8, depth-first order)."""
    keep, cp, nc = _cells(cells)
    b = _square(n, base)
    num = ctypes.c_int64(0)
    _check(_lib.dls_split_cells(n, flags, _u8(b), cp, nc, None, 0, ctypes.byref(num)), "dls_split_cells")
    out = np.zeros((num.value, n * n), dtype=np.uint8)
    if num.value:
        _check(_lib.dls_split_cells(n, flags, _u8(b), cp, nc, _u8(out), num.value, ctypes.byref(num)),
               "dls_split_cells")
    del keep
    return out


def dls_order_cost(n: int, flags: int, cells, prefixes):
    """(DFS steps, squares) of filling `cells` in this order over the host
    prefixes."""
    keep, cp, nc = _cells(cells)
    pre = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint8).reshape(-1, n * n))
    st, lv = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(_lib.dls_order_cost(n, flags, cp, nc, _u8(pre), len(pre), ctypes.byref(st), ctypes.byref(lv)),
           "dls_order_cost")
    del keep
    return int(st.value), int(lv.value)


def dls_hourglass_classes_async(n: int, d_designs, num: int, d_out, d_mult, cap: int, d_count,
                                d_status=None, stream=None) -> None:
    _check(_lib.dls_hourglass_classes_async(n, _ptr(d_designs), num, _ptr(d_out), _ptr(d_mult), cap,
                                            _ptr(d_count), _ptr(d_status), _stream(stream)),
           "dls_hourglass_classes_async")


def diagonal_cells(n: int) -> list:
    """Cells of both diagonals outside row 0, row-major."""
    return [c for c in range(n, n * n) if c // n == c % n or c // n + c % n == n - 1]


def hourglass_classes_gpu(n: int, stream=None):
    """Canonical hourglass designs of order n and their class powers,
    computed on the GPU from the diagonal designs (split on the host).
    Returns (designs [P, n*n] uint8, powers [P] uint32) sorted
    lexicographically."""
    import torch
    base = np.full(n * n, DLS_EMPTY, dtype=np.uint8)
    base[:n] = np.arange(n, dtype=np.uint8)
    designs = dls_split_cells(n, 0, base, diagonal_cells(n))
    dev = torch.device("cuda:0")
    d_des = torch.from_numpy(designs).to(dev)
    d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    d_st = torch.zeros(1, dtype=torch.int32, device=dev)
    cap = max(1024, len(designs))
    while True:
        d_out = torch.empty((cap, n * n), dtype=torch.uint8, device=dev)
        d_mult = torch.empty(cap, dtype=torch.int32, device=dev)
        d_st.zero_()
        dls_hourglass_classes_async(n, d_des, len(designs), d_out, d_mult, cap, d_cnt, d_st, stream)
        torch.cuda.synchronize()
        found = int(d_cnt.item())
        if found <= cap:
            break
        cap = found
    if int(d_st.item()) & ~8:
        raise DLSError(-4, f"hourglass classes: device status {int(d_st.item())}")
    out = d_out[:found].cpu().numpy()
    mult = d_mult[:found].cpu().numpy().view(np.uint32).copy()
    order = np.lexsort(out.T[::-1])
    return out[order], mult[order]


# --------------------------------------------------------------------------
# serving (continuous batching on the device): handles are plain ints
# --------------------------------------------------------------------------

def dls_server_create(max_jobs: int = 128, pool_bytes: int = 64 << 20, launch=None) -> int:
    """Handle of a new server (one long-running kernel for orders 4..9)."""
    h = ctypes.c_void_p()
    lc = _launch(launch)
    _check(_lib.dls_server_create(max_jobs, pool_bytes, None if lc is None else ctypes.byref(lc),
                                  ctypes.byref(h)), "dls_server_create")
    return int(h.value)


def dls_server_submit(server: int, n: int, flags: int, prefix, min_tasks: int) -> Optional[int]:
    """Ticket of the admitted request, or None when the server has no room
    now (DLS_EBUSY)."""
    p = _square(n, prefix)
    t = ctypes.c_int64(0)
    rc = _lib.dls_server_submit(ctypes.c_void_p(server), n, flags, _u8(p), min_tasks, ctypes.byref(t))
    if rc == DLS_EBUSY:
        return None
    _check(rc, "dls_server_submit")
    return int(t.value)


def dls_server_poll(server: int, ticket: int):
    """(done, count, (tick_start, tick_end)); count and ticks are None until done."""
    c = ctypes.c_uint64(0)
    ticks = (ctypes.c_uint64 * 2)()
    d = ctypes.c_int(0)
    _check(_lib.dls_server_poll(ctypes.c_void_p(server), ticket, ctypes.byref(c), ticks, ctypes.byref(d)),
           "dls_server_poll")
    if not d.value:
        return False, None, None
    return True, int(c.value), (int(ticks[0]), int(ticks[1]))


def dls_server_info(server: int) -> dict:
    b, pf, lc = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    sf = ctypes.c_int(0)
    _check(_lib.dls_server_info(ctypes.c_void_p(server), ctypes.byref(b), ctypes.byref(pf), ctypes.byref(sf),
                                ctypes.byref(lc)), "dls_server_info")
    return {"allocated_bytes": int(b.value), "pool_free": int(pf.value), "slots_free": int(sf.value),
            "launches": int(lc.value)}


def dls_server_waves(server: int) -> tuple:
    """(waves of the serving kernel running now, waves of its grid)."""
    live, grid = ctypes.c_int(0), ctypes.c_int(0)
    _check(_lib.dls_server_waves(ctypes.c_void_p(server), ctypes.byref(live), ctypes.byref(grid)),
           "dls_server_waves")
    return int(live.value), int(grid.value)


def dls_server_shared(server: int) -> int:
    """Subtrees handed between waves through the jobs' donation queues,
    over the requests retired so far."""
    k = ctypes.c_int64(0)
    _check(_lib.dls_server_shared(ctypes.c_void_p(server), ctypes.byref(k)), "dls_server_shared")
    return int(k.value)


def dls_server_destroy(server: int) -> None:
    _check(_lib.dls_server_destroy(ctypes.c_void_p(server)), "dls_server_destroy")


def dls_split_target(n: int, flags: int, base, min_tasks: int, max_depth: int = 24) -> np.ndarray:
    """Workunits of `base`, split breadth-first to at least min_tasks
    (or max_depth cells), [P, n*n] uint8."""
    b = _square(n, base)
    num = ctypes.c_int64(0)
    _check(_lib.dls_split_target(n, flags, _u8(b), min_tasks, max_depth, None, 0, ctypes.byref(num)),
           "dls_split_target")
    out = np.zeros((num.value, n * n), dtype=np.uint8)
    if num.value:
        _check(_lib.dls_split_target(n, flags, _u8(b), min_tasks, max_depth, _u8(out), num.value,
                                     ctypes.byref(num)), "dls_split_target")
    return out
