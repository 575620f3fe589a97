"""Partial squares on a given cell list (the incomplete squares of Sec. 5.3):
the GPU counts against the oracle's count of consistent assignments (exact
integers, tolerance 0), and the paper's N_10^30 for order 10."""
import numpy as np
import pytest

import oracle
from tests import golden_io

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()
import dls_workloads as workloads  # noqa: E402

E = 0xFF


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _left(n, cells):
    return [c for c in cells if 2 * (c % n) <= n - 1]


@pytest.mark.parametrize("n,k", [(4, 8), (5, 10), (6, 12), (7, 14), (8, 10), (9, 9)])
def test_row_major_cells_identity(n, k):
    base = oracle.identity_prefix(n)
    cells = list(range(n, n + k))
    got = dls.dls_count_cells(n, 0, cells, base[None])
    assert int(got[0]) == oracle.count_assignments(n, base, cells)


@pytest.mark.parametrize("n", [6, 8])
def test_vs_left_half_rows(n):
    base = oracle.identity_prefix(n)
    cells = _left(n, range(n, 3 * n))
    full = []
    for c in cells:
        full.append(c)
        full.append((c // n) * n + (n - 1 - c % n))
    got = dls.dls_count_cells(n, dls.DLS_VSYM, cells, base[None])
    assert int(got[0]) == oracle.count_assignments(n, base, full, vs=True)


def test_random_prefixes_and_cell_subsets():
    rng = workloads.SplitMix64(3053)
    for trial in range(12):
        n = 6 + rng.below(3)
        pre = workloads.random_prefix(n, n + rng.below(n), False, rng)
        empty = [c for c in range(n * n) if pre[c] == E]
        k = 4 + rng.below(min(10, len(empty) - 4))
        pick = sorted(workloads.sample_positions(len(empty), k, seed=trial))
        cells = [empty[i] for i in pick]
        got = dls.dls_count_cells(n, 0, cells, pre[None])
        assert int(got[0]) == oracle.count_assignments(n, pre, cells), (trial, n, cells)


def test_batch_on_device_with_expansion_and_plain():
    import torch
    n = 7
    pre, _ = dls.dls_split(n, 0, 8)
    cells = [c for c in range(n, 3 * n) if pre[0][c] == E]
    want = np.array([oracle.count_assignments(n, p, cells) for p in pre], dtype=np.uint64)
    dev = torch.device("cuda:0")
    d_pre = torch.from_numpy(pre).to(dev)
    pattern = (pre[0] != E).astype(np.uint8)
    for flags, launch in ((0, None), (0, {"expand_target": -1}), (dls.DLS_PLAIN, None)):
        d_cnt = torch.zeros(len(pre), dtype=torch.int64, device=dev)
        d_st = torch.zeros(1, dtype=torch.int32, device=dev)
        dls.dls_count_cells_async(n, flags, cells, pattern, d_pre, len(pre), d_cnt, d_st, None, launch)
        torch.cuda.synchronize()
        assert int(d_st.item()) == 0
        assert np.array_equal(d_cnt.cpu().numpy().view(np.uint64), want), (flags, launch)


def test_no_cells_counts_consistent_prefixes():
    n = 6
    good = oracle.identity_prefix(n)
    bad = good.copy()
    bad[n + 1] = 1                       # repeats the column-1 value of row 0
    got = dls.dls_count_cells(n, 0, [], np.stack([good, bad]))
    assert list(got) == [1, 0]


def test_order10_first_30_cells_row_major():
    # Sec. 5.3: N_10^30, the incomplete squares of order 10 formed by the first
    # 30 cells in row-major order with the first row fixed
    n = 10
    base = oracle.identity_prefix(n)
    got = dls.dls_count_cells(n, 0, list(range(n, 30)), base[None])
    assert int(got[0]) == golden_io.counts()[(10, "partial_rowmajor_30")]


def test_order10_first_32_cells_row_major():
    # Sec. 5.3: N_10^32 (about 11 s on one MI355X)
    n = 10
    base = oracle.identity_prefix(n)
    got = dls.dls_count_cells(n, 0, list(range(n, 32)), base[None])
    assert int(got[0]) == golden_io.counts()[(10, "partial_rowmajor_32")]
