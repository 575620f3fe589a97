"""Orders 11-16 on the GPU (the definition of Sec. 1 holds for every order;
the library takes 1 <= n <= 16).  Inputs: complete squares built by the
oracle's own search with seeded value orders, with 20, 40 or 64 cells emptied (for
vertical symmetry, left-half cells with their mirrors).  Every count is
compared with the oracle's, element by element, for both kernels and both
mask layouts of the persistent kernel (tolerance 0)."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import gpu_counts

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()
import dls_workloads as workloads  # noqa: E402

E = 0xFF
CASES = [(n, False) for n in range(11, 17)] + [(n, True) for n in (12, 14, 16)]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(n, vs, blanks, squares, seed):
    """`squares` complete squares (first row 0..n-1) with the same `blanks`
    cells emptied: one pattern, so one batch."""
    rng = workloads.SplitMix64(seed)
    full = []
    while len(full) < squares:
        vo = workloads.random_permutations(n, n * n, rng)
        try:     # a value order that leads the search astray is replaced
            sq = oracle.first_completion(n, oracle.identity_prefix(n), vo, vs=vs, node_limit=200_000)
        except ValueError:
            continue
        assert sq is not None and oracle.is_dls(n, sq, vs=vs)
        full.append(sq)
    mask = workloads.blank_cells(n, np.zeros(n * n, np.uint8), blanks, vs, rng) == E
    pre = np.stack(full)
    pre[:, mask] = E
    return pre


@pytest.fixture(scope="module")
def batches():
    out = {}
    for n, vs in CASES:
        for blanks in (20, 40, 64):
            k = blanks // 2 if vs else blanks      # vs: pairs
            pre = _batch(n, vs, k, 24, seed=1000 * n + 10 * blanks + vs)
            out[(n, vs, blanks)] = (pre, oracle.count_many(n, pre, vs=vs))
    return out


@pytest.mark.parametrize("n,vs", CASES)
@pytest.mark.parametrize("blanks", [20, 40, 64])
@pytest.mark.parametrize("kernel", ["plain", "vgpr", "lds"])
def test_near_complete_squares_match_oracle(batches, n, vs, blanks, kernel):
    pre, want = batches[(n, vs, blanks)]
    assert np.all(want >= 1)                    # each square is its own completion
    flags = dls.DLS_VSYM if vs else 0
    launch = None if kernel == "plain" else {"lds_masks": 1 if kernel == "lds" else -1}
    c, st = gpu_counts(dls, n, flags, pre, plain=kernel == "plain", launch=launch)
    assert st == 0
    assert np.array_equal(c, want), (n, vs, blanks, kernel)


@pytest.mark.parametrize("n", [11, 13, 16])
def test_large_order_mixed_patterns_through_host_api(batches, n):
    # dls_count groups prefixes by pattern; a broken prefix counts 0
    a, wa = batches[(n, False, 20)]
    b, wb = batches[(n, False, 40)]
    pre = np.concatenate([a[:8], b[:8]])
    bad = a[0].copy()
    bad[n] = bad[n + 1] if bad[n + 1] != E else 0   # repeat a value in row 1 (or any change)
    pre = np.concatenate([pre, bad[None]])
    got = dls.dls_count(n, 0, pre)
    want = np.concatenate([wa[:8], wb[:8], oracle.count_many(n, bad[None])])
    assert np.array_equal(got, want)
