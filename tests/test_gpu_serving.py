"""Serving: requests of different orders, flags and prefix sizes run
concurrently on the GPU; each count must be the same alone and in the mix,
and equal to the oracle's (exact integers: tolerance 0)."""
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


def _requests(count, seed, k_range=None):
    from paper_1709_02599_amd.serve import Request
    jobs = dls_workloads.job_stream(count, rate=1000.0, seed=seed, k_range=k_range)
    return [Request(j.jid, j.n, j.vs, j.prefix, j.arrival) for j in jobs]


@pytest.mark.parametrize("host_split", [False, True])
def test_mix_equals_solo_equals_oracle(host_split):
    from paper_1709_02599_amd.serve import Server
    reqs = _requests(40, seed=5)
    srv = Server(slots=4, min_tasks=2048, host_split=host_split)
    mix = srv.run(reqs, realtime=False)
    assert [r.rid for r in mix] == [q.rid for q in reqs]
    for q, r in zip(reqs, mix):
        flags = dls.DLS_VSYM if q.vs else 0
        solo = int(dls.dls_count(q.n, flags, q.prefix[None])[0])
        assert r.count == solo, (q.rid, q.n, q.vs)
        if solo <= 3_000_000:
            assert solo == oracle.count(q.n, q.prefix, vs=q.vs), (q.rid, q.n, q.vs)
        if q.vs and q.n % 2:
            assert solo == 0


def test_realtime_arrivals_and_admission_by_memory():
    from paper_1709_02599_amd.serve import Server, latency_stats
    reqs = _requests(16, seed=7)
    # host-split requests of about 1024 workunits: a 1 MiB budget admits one
    # at a time mostly
    srv = Server(slots=2, mem_budget=1 << 20, min_tasks=1024, host_split=True)
    res = srv.run(reqs, realtime=True)
    ref = Server(slots=4).run(reqs, realtime=False)
    assert [a.count for a in res] == [b.count for b in ref]
    st = latency_stats(res)
    assert st["n"] == 16 and st["p99_ms"] >= st["p50_ms"] > 0
    assert sum(v["n"] for v in st["per_order"].values()) == 16
