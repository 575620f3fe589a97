"""The allocation-free entry point (dls_count_async_noalloc): its counts equal
those of dls_count_async_ex bit for bit, on two calls in a row (the second
with a smaller input, which reuses the static scratch the first left
behind), for both kernels; a batch that does not fit is refused on the
host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()

E = 0xFF


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(n, flags, pre, launch=None):
    """Counts of the existing entry point and of the allocation-free one,
    on the same device prefixes; returns (counts_ex, counts_noalloc,
    status_ex, status_noalloc)."""
    import torch
    dev = torch.device("cuda:0")
    num = len(pre)
    pattern = (pre[0] != E).astype(np.uint8)
    d_pre = torch.from_numpy(np.ascontiguousarray(pre)).to(dev)
    c_ex = torch.full((num,), -1, dtype=torch.int64, device=dev)
    c_na = torch.full((num,), -2, dtype=torch.int64, device=dev)
    s_ex = torch.zeros(1, dtype=torch.int32, device=dev)
    s_na = torch.zeros(1, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    dls.dls_count_async_ex(n, flags, pattern, d_pre, num, c_ex, s_ex, st, launch)
    dls.dls_count_async_noalloc(n, flags, pattern, d_pre, num, c_na, s_na, st, launch)
    torch.cuda.synchronize()
    return (c_ex.cpu().numpy().view(np.uint64), c_na.cpu().numpy().view(np.uint64),
            int(s_ex.item()), int(s_na.item()))


@pytest.mark.parametrize("flags", [0, dls.DLS_PLAIN])
def test_noalloc_equals_existing_entry_point_twice(flags):
    # first call: the order-8 workload with symmetry breaking (2 819 311
    # prefixes); second call: the order-7 diagonal split (2 016 prefixes,
    # deepened on the device inside the static array)
    big, _ = dls.dls_split(8, dls.DLS_SYMBREAK, 26)
    small, _ = dls.dls_split(7, 0, 11)
    for n, pre in ((8, big), (7, small)):
        a, b, sa, sb = _both(n, flags, pre)
        assert sa == 0 and sb == 0
        assert np.array_equal(a, b), (n, flags)
    assert int(b.sum()) == 171200                   # order 7, first row fixed


def test_noalloc_tuned_launch_and_donation():
    pre, _ = dls.dls_split(8, dls.DLS_SYMBREAK, 26)
    launch = {"block": 256, "blocks_per_cu": 16, "refill_every": 128, "order_variant": 5,
              "chunk_min": 16, "lds_masks": -1, "refill_min": 1}
    a, b, sa, sb = _both(8, 0, pre, launch)
    assert sa == sb == 0 and np.array_equal(a, b)
    # a few huge prefixes with the expansion off: donation across the chip
    # through the donated-record slots of the static array
    few, _ = dls.dls_split(8, 0, 6)
    a, b, sa, sb = _both(8, 0, few[:40], {"expand_target": -1, "steal_depth": 8})
    assert sa == sb == 0 and np.array_equal(a, b)


def test_noalloc_refuses_what_does_not_fit():
    import torch
    dev = torch.device("cuda:0")
    d = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.zeros(1, dtype=torch.int32, device=dev)
    # 16 M order-16 prefixes would need 1.3 GB of task records: refused on
    # the host before any launch (the pointers are never read)
    with pytest.raises(dls.DLSError) as ei:
        dls.dls_count_async_noalloc(16, 0, None, d, 1 << 24, d, s, None, None)
    assert ei.value.code == -2                      # DLS_ERANGE
    with pytest.raises(dls.DLSError) as ei:
        dls.dls_count_async_noalloc(7, 0, None, d, 1, d, None, None, None)
    assert ei.value.code == -1                      # d_status is required
    with pytest.raises(dls.DLSError) as ei:
        dls.dls_count_async_noalloc(7, 0, None, d, 1, d, s, None, {"time_kernel": 1})
    assert ei.value.code == -1
