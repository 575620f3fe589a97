"""GPU tests of launch plumbing: HIP graph capture and replay of a counting
step, fill-order variants, per-kernel event timing and the device weighted
reduction.  Every count is compared with the oracle's (tolerance 0)."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import gpu_counts

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()

E = 0xFF


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_split(n, depth):
    base = oracle.identity_prefix(n)
    order = oracle.fill_order(n, list(range(n)))
    return oracle.assignments(n, base, order[:depth])


@pytest.fixture(scope="module")
def order7():
    pre, _ = dls.dls_split(7, 0, 8)
    opre = _oracle_split(7, 8)
    assert np.array_equal(pre, opre)
    return pre, oracle.count_many(7, opre)


@pytest.mark.parametrize("flags", [0, 4])          # persistent, plain
def test_graph_replays_recount_every_time(order7, flags):
    import torch
    from paper_1709_02599_amd.graphs import CountStep
    pre, want = order7
    dev = torch.device("cuda:0")
    num = len(pre)
    d_pre = torch.from_numpy(pre).to(dev)
    d_cnt = torch.zeros(num, dtype=torch.int64, device=dev)
    d_st = torch.zeros(1, dtype=torch.int32, device=dev)
    mult = (np.arange(num) % 5 + 1).astype(np.int32)          # arbitrary weights
    d_mult = torch.from_numpy(mult).to(dev)
    pattern = (pre[0] != E).astype(np.uint8)
    step = CountStep(7, flags, pattern, d_pre, num, d_cnt, d_st, d_mult).capture()
    want_total = int((want.astype(np.int64) * mult).sum())
    other = torch.zeros(1, dtype=torch.int64, device=dev)
    for rep in range(4):
        # eager work between replays: clobber the outputs, run an unrelated
        # eager count of other prefixes on the default stream, synchronise
        d_cnt.fill_(-1)
        step.total.fill_(-7)
        c, st = gpu_counts(dls, 7, 0, pre[rep::7])
        assert st == 0 and np.array_equal(c, want[rep::7])
        other.add_(1)
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        got = d_cnt.cpu().numpy().view(np.uint64)
        assert int(d_st.item()) == 0
        assert np.array_equal(got, want), f"replay {rep}"
        assert int(step.total.item()) == want_total, f"replay {rep}"
    # eager issue of the same step agrees too
    step.eager()
    torch.cuda.synchronize()
    assert int(step.total.item()) == want_total


def test_capture_without_prior_call_is_refused():
    import torch
    dev = torch.device("cuda:0")
    pre = oracle.identity_prefix(6)[None, :]
    d_pre = torch.from_numpy(pre).to(dev)
    d_cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.Stream()                 # never used by the library
    x = torch.zeros(1, dtype=torch.int64, device=dev)
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        with pytest.raises(dls.DLSError) as ei:
            dls.dls_count_async_ex(6, 0, None, d_pre, 1, d_cnt, None, s, None)
        x.add_(1)
    assert ei.value.code == dls.DLS_ECAPTURE
    g.replay()
    torch.cuda.synchronize()
    assert int(x.item()) == 1
    # the same call outside capture works
    dls.dls_count_async_ex(6, 0, None, d_pre, 1, d_cnt, None, s, None)
    torch.cuda.synchronize()
    assert int(d_cnt.item()) == oracle.count(6, oracle.identity_prefix(6))


@pytest.mark.parametrize("variant", range(8))
def test_order_variants_count_the_same(order7, variant):
    pre, want = order7
    c, st, steps = gpu_counts(dls, 7, 0, pre, launch={"order_variant": variant}, steps=True)
    assert st == 0 and np.array_equal(c, want)
    assert steps > 0


def test_order_variants_change_the_work(order7):
    pre, _ = order7
    steps = {v: gpu_counts(dls, 7, 0, pre, launch={"order_variant": v}, steps=True)[2]
             for v in range(8)}
    assert len(set(steps.values())) > 1, steps


def test_kernel_timing_counts_launches():
    import torch
    pre, _ = dls.dls_split(7, 0, 11)
    dev = torch.device("cuda:0")
    d_pre = torch.from_numpy(pre).to(dev)
    d_cnt = torch.zeros(len(pre), dtype=torch.int64, device=dev)
    s = torch.cuda.current_stream()
    pattern = (pre[0] != E).astype(np.uint8)
    for k in range(3):
        dls.dls_count_async_ex(7, 0, pattern, d_pre, len(pre), d_cnt, None, s,
                               {"time_kernel": 1})
    dls.dls_count_async_ex(7, 0, pattern, d_pre, len(pre), d_cnt, None, s, None)   # untimed
    torch.cuda.synchronize()
    ms, launches = dls.dls_kernel_time_ms(s)
    assert launches == 3 and 0.0 < ms < 1000.0
    with pytest.raises(dls.DLSError):
        dls.dls_kernel_time_ms(s)                       # tally was reset


def test_reduce_weighted_matches_host():
    import torch
    rng = np.random.default_rng(5)
    dev = torch.device("cuda:0")
    for num in (0, 1, 255, 256, 257, 100_003, 3_000_001):
        c = rng.integers(0, 1 << 40, size=num, dtype=np.int64)
        m = rng.integers(0, 200, size=num, dtype=np.int32)
        d_c = torch.from_numpy(c).to(dev)
        d_m = torch.from_numpy(m).to(dev)
        out = torch.full((1,), -1, dtype=torch.int64, device=dev)
        dls.dls_reduce_weighted(d_c, d_m, num, out)
        out1 = torch.full((1,), -1, dtype=torch.int64, device=dev)
        dls.dls_reduce_weighted(d_c, None, num, out1)
        torch.cuda.synchronize()
        want = int((c.astype(object) * m.astype(object)).sum()) % (1 << 64)
        assert int(out.item()) % (1 << 64) == want, num
        assert int(out1.item()) == int(c.astype(object).sum()), num


def test_host_order_cost_equals_device_step_count(order7):
    # the kernels' instrumented DFS step count (down + up) is twice the host
    # cost of the same fill order (expansion off: its levels are not steps)
    pre, _ = order7
    pattern = (pre[0] != E).astype(np.uint8)
    for v in (0, 5):
        _, st, steps = gpu_counts(dls, 7, 0, pre, launch={"order_variant": v, "expand_target": -1},
                                  steps=True)
        order = dls.dls_order_variant(7, 0, pattern, v)
        host_steps, _ = dls.dls_order_cost(7, 0, order, pre)
        assert st == 0 and steps == 2 * host_steps, v


def test_captured_graph_survives_a_larger_eager_batch_on_its_stream(order7):
    # A captured step keeps the addresses of its stream's scratch; a later
    # uncaptured call on the same stream with a larger batch must not free
    # them (the library retires outgrown buffers of captured streams).
    import torch
    from paper_1709_02599_amd.graphs import CountStep
    pre, want = order7
    dev = torch.device("cuda:0")
    small = pre[:300].copy()
    d_pre = torch.from_numpy(small).to(dev)
    d_cnt = torch.zeros(len(small), dtype=torch.int64, device=dev)
    d_st = torch.zeros(1, dtype=torch.int32, device=dev)
    pattern = (small[0] != E).astype(np.uint8)
    step = CountStep(7, 0, pattern, d_pre, len(small), d_cnt, d_st,
                     launch=dls.DlsLaunch(expand_target=4096)).capture()
    big_pre, _ = dls.dls_split(7, 0, 11)
    big_want = oracle.count_many(7, big_pre)
    d_big = torch.from_numpy(big_pre).to(dev)
    for rep in range(3):
        # larger batch, larger expansion target: both outgrow the captured buffers
        d_bc = torch.zeros(len(big_pre), dtype=torch.int64, device=dev)
        dls.dls_count_async_ex(7, 0, (big_pre[0] != E).astype(np.uint8), d_big, len(big_pre), d_bc, None,
                               step.stream, dls.DlsLaunch(expand_target=8192 << rep))
        step.stream.synchronize()
        assert dls.dls_stream_status(step.stream) == 0
        assert np.array_equal(d_bc.cpu().numpy().view(np.uint64), big_want)
        d_cnt.fill_(-1)
        torch.cuda.synchronize()
        step.replay()
        torch.cuda.synchronize()
        assert int(d_st.item()) == 0
        assert np.array_equal(d_cnt.cpu().numpy().view(np.uint64), want[:300]), f"replay {rep}"


def test_host_order_cost_equals_device_step_count_order8():
    # order 8 runs the two-word diagonal form with a sentinel level past the
    # last; its steps onto and off the sentinel are not DFS steps
    import torch
    import dls_workloads as workloads
    pre, _ = dls.dls_split(8, 0, 12)
    pre = pre[workloads.sample_positions(len(pre), 3000, seed=12)]
    pattern = (pre[0] != E).astype(np.uint8)
    want = oracle.count_many(8, pre)
    dev = torch.device("cuda:0")
    d_pre = torch.from_numpy(pre).to(dev)
    for v in (0, 5):
        order = dls.dls_order_variant(8, 0, pattern, v)
        host_steps, leaves = dls.dls_order_cost(8, 0, order, pre)
        assert leaves == int(want.sum())
        for launch in ({"order_variant": v, "expand_target": -1},
                       {"order_variant": v, "expand_target": -1, "steal_depth": 6, "refill_every": 8}):
            d_cnt = torch.zeros(len(pre), dtype=torch.int64, device=dev)
            d_st = torch.zeros(1, dtype=torch.int32, device=dev)
            d_steps = torch.zeros(2, dtype=torch.int64, device=dev)
            dls.dls_count_async_stats(8, 0, pattern, d_pre, len(pre), d_cnt, d_st, None, launch, d_steps)
            torch.cuda.synchronize()
            assert int(d_st.item()) == 0
            assert np.array_equal(d_cnt.cpu().numpy().view(np.uint64), want), launch
            assert int(d_steps[0].item()) == 2 * host_steps, launch
            assert int(d_steps[1].item()) >= int(d_steps[0].item())
