"""Serving: requests of different orders, flags and prefix sizes batched
continuously on the GPU by the library's serving kernel (one long-running
kernel for every order and flags, fed through a job ring it polls).  Each
count must be the same alone and in the mix and equal the oracle's (exact
integers: tolerance 0); requests must run on the device at the same time;
admission must follow the servers' real allocation."""
import collections
import time

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()
import dls_workloads  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _requests(count, seed, k_range=None, rate=1000.0):
    from paper_1709_02599_amd.serve import Request
    jobs = dls_workloads.job_stream(count, rate=rate, seed=seed, k_range=k_range)
    return [Request(j.jid, j.n, j.vs, j.prefix, j.arrival) for j in jobs]


def _oracle(reqs):
    """The oracle's count of every request (grouped by order and flags)."""
    groups = collections.defaultdict(list)
    for q in reqs:
        groups[(q.n, q.vs)].append(q)
    out = {}
    for (n, vs), qs in groups.items():
        c = oracle.count_many(n, np.stack([q.prefix for q in qs]), vs=vs)
        for q, v in zip(qs, c):
            out[q.rid] = int(v)
    return out


def test_every_count_equals_the_oracle_in_the_mix():
    # requests whose counts the oracle finishes in seconds (k in [12, 20])
    from paper_1709_02599_amd.serve import Server
    reqs = _requests(64, seed=5, k_range=(12, 20))
    want = _oracle(reqs)
    with Server(min_tasks=512) as srv:
        res = srv.run(reqs, realtime=False)
    assert [r.rid for r in res] == [q.rid for q in reqs]
    for q, r in zip(reqs, res):
        assert r.count == want[q.rid], (q.rid, q.n, q.vs)
        if q.vs and q.n % 2:
            assert r.count == 0
    assert any(want.values())


def test_mix_equals_solo_and_jobs_overlap_on_the_device():
    # the workload's own prefix sizes (k in [N, 3N]): every count equals the
    # count of the same request served alone; several requests are counted
    # on the device at the same time (device timestamps of first chunk and
    # last piece)
    from paper_1709_02599_amd.serve import Server
    reqs = _requests(40, seed=7)
    with Server(min_tasks=2048) as srv:
        mix = srv.run(reqs, realtime=False)
        solo = [srv.run([q], realtime=False)[0] for q in reqs]
        info = srv.info()
    for q, a, b in zip(reqs, mix, solo):
        assert a.count == b.count, (q.rid, q.n, q.vs)
        # the plain count API agrees too
        assert a.count == int(dls.dls_count(q.n, dls.DLS_VSYM if q.vs else 0, q.prefix[None])[0])
    small = [q for q, a in zip(reqs, mix) if a.count <= 100_000]
    want = _oracle(small)
    for q in small:
        assert [r for r in mix if r.rid == q.rid][0].count == want[q.rid]
    # requests were served by a running kernel, not one launch each
    assert info["launches"] < len(reqs)


def test_requests_run_on_the_device_at_the_same_time():
    # heavier requests (order 8, 6-8 cells beyond the first row) admitted
    # together: their device intervals (job taken up -> last piece done)
    # overlap, and each count equals the request's count alone
    from paper_1709_02599_amd.serve import Request, Server, max_concurrency, overlapping_pairs
    jobs = dls_workloads.job_stream(12, rate=1000.0, seed=11, orders=(8,), vs_choices=(False,), k_range=(6, 8))
    reqs = [Request(j.jid, j.n, j.vs, j.prefix, 0.0) for j in jobs]
    with Server(min_tasks=2048) as srv:
        mix = srv.run(reqs, realtime=False)
        assert srv.peak_in_flight >= 2
    solo = dls.dls_count(8, 0, np.stack([q.prefix for q in reqs]))
    assert [r.count for r in mix] == [int(c) for c in solo]
    busy = [r for r in mix if r.dev_end > 0]
    assert len(busy) >= 2
    assert max_concurrency(mix) >= 2, [(r.dev_start, r.dev_end) for r in busy]
    assert overlapping_pairs(mix) >= 1


def test_admission_follows_the_pool():
    # a pool of 256 KiB (4 096 workunits of order 8) and 4 ring slots: at
    # most a few requests fit at once, the rest wait for room (DLS_EBUSY); the
    # peak of pool bytes in use never exceeds the pool; every count is exact
    from paper_1709_02599_amd.serve import Server
    reqs = _requests(48, seed=5, k_range=(12, 20))
    want = _oracle(reqs)
    with Server(pool_bytes=256 << 10, max_jobs=4, min_tasks=256) as srv:
        res = srv.run(reqs, realtime=False)
        assert srv.busy_answers > 0
        assert 0 < srv.peak_pool_used <= 256 << 10
        info = srv.info()
        assert info["pool_free"] == 256 << 10 and info["slots_free"] == 4     # all retired
        assert info["allocated_bytes"] >= 256 << 10
    for q, r in zip(reqs, res):
        assert r.count == want[q.rid]


def test_realtime_arrivals_and_latency_stats():
    from paper_1709_02599_amd.serve import Server, latency_stats
    reqs = _requests(24, seed=9, k_range=(12, 20), rate=400.0)
    want = _oracle(reqs)
    with Server(min_tasks=512) as srv:
        res = srv.run(reqs, realtime=True)
    assert [r.count for r in res] == [want[q.rid] for q in reqs]
    st = latency_stats(res)
    assert st["n"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0
    assert sum(v["n"] for v in st["per_order"].values()) == 24
    assert all(r.done >= r.admitted >= r.arrival for r in res)


def test_server_leaves_when_idle_and_comes_back():
    # the kernel leaves after 50 ms without work; the next request launches it again
    n = 7
    h = dls.dls_server_create(max_jobs=8, pool_bytes=1 << 20)
    try:
        p = oracle.identity_prefix(n)
        counts = []
        for rep in range(2):
            t = dls.dls_server_submit(h, n, 0, p, 256)
            assert t is not None
            t_end = time.time() + 30
            while True:
                done, c, ticks = dls.dls_server_poll(h, t)
                if done:
                    break
                assert time.time() < t_end, "request not done"
                time.sleep(0.0005)
            counts.append(c)
            assert ticks[1] >= ticks[0] > 0
            time.sleep(0.2)                          # longer than the idle limit
        assert counts == [171200, 171200]            # order 7, first row fixed
        assert dls.dls_server_info(h)["launches"] >= 2
        # an inconsistent prefix is done at once with count 0
        bad = p.copy()
        bad[n] = 0                                   # (1,0) repeats the value of (0,0)
        t = dls.dls_server_submit(h, n, 0, bad, 256)
        assert dls.dls_server_poll(h, t)[:2] == (True, 0)
        with pytest.raises(dls.DLSError):
            dls.dls_server_poll(h, t)                # retired
        # vertical symmetry at an odd order: 0 at once
        t = dls.dls_server_submit(h, n, dls.DLS_VSYM, p, 256)
        assert dls.dls_server_poll(h, t)[:2] == (True, 0)
    finally:
        dls.dls_server_destroy(h)


def test_server_argument_errors():
    h = dls.dls_server_create(max_jobs=2, pool_bytes=4096)
    try:
        with pytest.raises(dls.DLSError):
            dls.dls_server_submit(h, 10, 0, oracle.identity_prefix(10), 16)   # beyond the served orders
        with pytest.raises(dls.DLSError):
            dls.dls_server_submit(h, 8, dls.DLS_SYMBREAK, oracle.identity_prefix(8), 16)
        # a split larger than the whole pool (4 KiB = 64 workunits of order 8)
        with pytest.raises(dls.DLSError) as ei:
            dls.dls_server_submit(h, 8, 0, oracle.identity_prefix(8), 100_000)
        assert ei.value.code == -2
    finally:
        dls.dls_server_destroy(h)


def _wait(h, ticket, limit_s):
    t_end = time.time() + limit_s
    while True:
        done, c, ticks = dls.dls_server_poll(h, ticket)
        if done:
            return c, ticks
        assert time.time() < t_end, "request not done"
        time.sleep(0.0005)


def test_grid_stays_whole_while_a_long_job_runs():
    # A long request in one workunit keeps one wave busy (with the handing
    # of subtrees between waves off); the
    # rest of the grid has nothing to take for longer than the idle limit
    # (50 ms) but stays, so requests submitted meanwhile are served by the
    # whole grid and finish long before the long one.  Once nothing runs,
    # the grid leaves as a whole.
    n = 8
    units = dls.dls_split_target(n, 0, oracle.identity_prefix(n), 400, 24)
    counts = dls.dls_count(n, 0, units)
    pick = int(np.argmin(np.abs(np.log(np.maximum(counts, 1).astype(np.float64)) - np.log(2e7))))
    long_prefix, long_count = units[pick], int(counts[pick])
    assert 5e6 <= long_count <= 5e7, long_count
    # orders 7 and 8: their oracle counts take well under a second
    from paper_1709_02599_amd.serve import Request
    small = [Request(j.jid, j.n, j.vs, j.prefix, 0.0)
             for j in dls_workloads.job_stream(16, 1000.0, seed=13, orders=(7, 8), k_range=(14, 20))]
    want = _oracle(small)
    # one workunit and no handing of subtrees between waves: the long job
    # keeps the one wave that took it
    h = dls.dls_server_create(max_jobs=64, pool_bytes=16 << 20, launch={"steal_depth": -1})
    try:
        t_long = dls.dls_server_submit(h, n, 0, long_prefix, 1)
        t0 = time.time()
        time.sleep(0.2)
        live, grid = dls.dls_server_waves(h)
        done_early = dls.dls_server_poll(h, t_long)[0]
        print(f"long job: count {long_count}; after 0.2 s: {live}/{grid} waves live, done={done_early}", flush=True)
        assert not done_early, "the long job must outlast the idle limit for this test to mean anything"
        assert live == grid
        tickets = [(q, dls.dls_server_submit(h, q.n, dls.DLS_VSYM if q.vs else 0, q.prefix, 512)) for q in small]
        ends = []
        for q, t in tickets:
            c, ticks = _wait(h, t, 30)
            assert c == want[q.rid], (q.rid, q.n, q.vs)
            ends.append(ticks[1])
        t_small = time.time() - t0
        c, ticks = _wait(h, t_long, 120)
        t_all = time.time() - t0
        print(f"small requests done after {t_small:.3f} s, long one after {t_all:.3f} s", flush=True)
        assert c == long_count
        assert max(e for e in ends if e) < ticks[1]
        assert dls.dls_server_info(h)["launches"] == 1
        time.sleep(0.3)                  # longer than the idle limit: the grid leaves as a whole
        assert dls.dls_server_waves(h)[0] == 0
    finally:
        dls.dls_server_destroy(h)


def _serve_one(n, flags, prefix, min_tasks, launch=None):
    """(count, device seconds, subtrees handed between waves) of one request
    served alone by a fresh server."""
    h = dls.dls_server_create(max_jobs=4, pool_bytes=4 << 20, launch=launch)
    try:
        t = dls.dls_server_submit(h, n, flags, prefix, min_tasks)
        c, ticks = _wait(h, t, 120)
        return c, (ticks[1] - ticks[0]) * 1e-8, dls.dls_server_shared(h)
    finally:
        dls.dls_server_destroy(h)


def _order8_unit(lo, hi):
    """A workunit of the order-8 first-row split whose count (batch path)
    lies in [lo, hi], and that count."""
    units = dls.dls_split_target(8, 0, oracle.identity_prefix(8), 400, 24)
    counts = dls.dls_count(8, 0, units)
    target = np.sqrt(lo * hi)
    k = int(np.argmin(np.abs(np.log(np.maximum(counts, 1).astype(np.float64)) - np.log(target))))
    assert lo <= counts[k] <= hi, int(counts[k])
    return units[k], int(counts[k])


def test_one_request_is_shared_across_waves():
    # a request of one workunit with handing between waves on (steal_depth
    # 8): its wave's lanes share it, and waves without work take subtrees
    # those lanes hand on through the job's donation queue.  The count
    # equals the oracle's (exact), and subtrees were handed on.
    base = oracle.identity_prefix(8)
    units = dls.dls_split_target(8, 0, base, 400, 24)
    deeper = dls.dls_split_target(8, 0, units[0], 64, 24)
    counts = dls.dls_count(8, 0, deeper)
    k = int(np.argmin(np.abs(np.log(np.maximum(counts, 1).astype(np.float64)) - np.log(1.5e5))))
    prefix = deeper[k]
    want = oracle.count(8, prefix)
    assert 2e4 <= want <= 1e6, want
    c, secs, shared = _serve_one(8, 0, prefix, 1, launch={"steal_depth": 8})
    print(f"count {c}, {secs * 1e3:.2f} ms on the device, {shared} subtrees handed between waves", flush=True)
    assert c == want
    assert shared > 0


@pytest.mark.parametrize("steal", [0, -1, 2, 16])
def test_sharing_across_waves_default_off_and_shallow(steal):
    # the same heavy request in one workunit with the default (no handing
    # between waves), handing off, from all but the last two levels (many
    # small subtrees: the job's ring of 2048 records is reused many times
    # over) and from 16 levels up: the count is unchanged
    prefix, count = _order8_unit(1e6, 3e7)
    c, secs, shared = _serve_one(8, 0, prefix, 1, launch={"steal_depth": steal} if steal else None)
    print(f"steal_depth {steal}: count {c}, {secs * 1e3:.2f} ms, {shared} subtrees handed on", flush=True)
    assert c == count
    if steal <= 0:
        assert shared == 0
    else:
        assert shared > 0


def test_workunits_spread_over_the_grid():
    # a request of 64 workunits: a wave takes one at a time (the job's
    # workunits over twice the grid's waves, at least one), so 64 waves
    # share the work and the request finishes well before the same request
    # in one workunit does (one wave); both counts are exact
    prefix, count = _order8_unit(1e6, 3e7)
    c64, t64, _ = _serve_one(8, 0, prefix, 64)
    c1, t1, _ = _serve_one(8, 0, prefix, 1)
    print(f"count {count}: 64 workunits {t64 * 1e3:.2f} ms, one workunit {t1 * 1e3:.2f} ms", flush=True)
    assert c64 == c1 == count
    assert t64 < 0.5 * t1
