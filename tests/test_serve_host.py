"""Host side of the serving loop, on the CPU: the statistics it reports over
device intervals and latencies (checked against brute force and numpy), and
the serving entry points' argument errors that need no device."""
import itertools

import numpy as np
import pytest

from tests.needs_lib import load as _load_dls

dls = _load_dls()
from paper_1709_02599_amd.serve import Result, latency_stats, max_concurrency, overlapping_pairs  # noqa: E402


def _results(rng, k, with_idle=True):
    """k results with distinct integer device times; some without device work."""
    times = rng.choice(10_000, size=2 * k, replace=False)
    out = []
    for i in range(k):
        s, e = sorted(times[2 * i:2 * i + 2])
        r = Result(i, 0, arrival=0.001 * i, admitted=0.001 * i, done=0.001 * i + 1e-4 * (e - s), n=7 + i % 3,
                   dev_start=int(s), dev_end=int(e))
        if with_idle and i % 5 == 4:
            r.dev_start = r.dev_end = 0  # done without search
        out.append(r)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_overlaps_and_concurrency_equal_brute_force(seed):
    rng = np.random.default_rng(seed)
    res = _results(rng, 24)
    iv = [(r.dev_start, r.dev_end) for r in res if r.dev_end > 0]
    pairs = sum(1 for (a, b), (c, d) in itertools.combinations(iv, 2) if a < d and c < b)
    assert overlapping_pairs(res) == pairs
    peak = max(sum(1 for s, e in iv if s <= t < e) for t, _ in iv)
    assert max_concurrency(res) == peak


def test_disjoint_and_nested_intervals():
    def r(i, s, e):
        return Result(i, 0, 0.0, 0.0, 0.0, dev_start=s, dev_end=e)
    chain = [r(0, 1, 2), r(1, 2, 3), r(2, 3, 4)]          # touching ends do not overlap
    assert overlapping_pairs(chain) == 0 and max_concurrency(chain) == 1
    nest = [r(0, 1, 100), r(1, 2, 50), r(2, 3, 10), r(3, 60, 70)]
    assert overlapping_pairs(nest) == 4 and max_concurrency(nest) == 3
    assert overlapping_pairs([]) == 0 and max_concurrency([]) == 0


def test_latency_stats_match_numpy():
    rng = np.random.default_rng(3)
    res = _results(rng, 40, with_idle=False)
    st = latency_stats(res)
    lat = np.array([r.latency for r in res])
    assert st["n"] == 40
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert st["mean_ms"] == pytest.approx(lat.mean() * 1e3)
    for n, v in st["per_order"].items():
        sub = np.array([r.latency for r in res if r.n == int(n)])
        assert v["n"] == len(sub) and v["p99_ms"] == pytest.approx(np.percentile(sub, 99) * 1e3)
    assert sum(v["n"] for v in st["per_order"].values()) == 40


def test_server_entry_points_reject_a_null_server():
    for call in (lambda: dls.dls_server_shared(0), lambda: dls.dls_server_waves(0),
                 lambda: dls.dls_server_info(0), lambda: dls.dls_server_destroy(0)):
        with pytest.raises(dls.DLSError) as ei:
            call()
        assert ei.value.code == -1
