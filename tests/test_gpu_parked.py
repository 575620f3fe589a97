"""GPU regression test of the persistent kernel's parked lanes.  Every lane
of a wave takes the DFS step on every iteration; a lane whose task has ended,
or started without candidates, is parked at its start level and must change
nothing until it is refilled.  Batches that mix live tasks with tasks that
are dead at their start (inconsistent or without candidates) are counted
under both mask layouts, extreme refill cadences and tiny grids; every count
must equal the oracle's (tolerance 0).  Inputs: all 128 order-6 DLS with the
identity first row (enumerated by the oracle), with k cells blanked and, in
half of the rows, one assigned cell set to a seeded random value."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import gpu_counts

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()

E = 0xFF
N = 6


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def squares():
    base = oracle.identity_prefix(N)
    full = oracle.assignments(N, base, list(range(N, N * N)))
    assert len(full) == 128 and all(oracle.is_dls(N, s) for s in full[:8])
    return full


def _batch(full, blank, seed):
    rng = np.random.default_rng(seed)
    live = full.copy()
    live[:, blank] = E
    kept = [c for c in range(N, N * N) if c not in blank]
    dead = live.copy()
    for t in range(len(dead)):
        dead[t, kept[rng.integers(len(kept))]] = rng.integers(0, N)
    batch = np.concatenate([live, dead])
    batch = batch[rng.permutation(len(batch))]
    return np.ascontiguousarray(np.tile(batch, (6, 1)))


LAUNCHES = [
    {},
    {"expand_target": -1, "refill_every": 1, "block": 64, "blocks_per_cu": 1},
    {"expand_target": -1, "refill_every": 2, "block": 64, "blocks_per_cu": 1, "lds_masks": 1},
    {"expand_target": -1, "refill_every": 3, "chunk_min": 1, "lds_masks": -1},
    {"refill_every": 5, "lds_masks": 1},
    {"expand_target": -1, "steal_depth": 4, "block": 64, "blocks_per_cu": 1, "lds_masks": 1},
]


@pytest.mark.parametrize("k", [4, 12, 22])
@pytest.mark.parametrize("li", range(len(LAUNCHES)))
def test_parked_lanes_change_nothing(squares, k, li):
    rng = np.random.default_rng(100 + k)
    blank = sorted(rng.choice(np.arange(2 * N, N * N), size=k, replace=False).tolist())
    batch = _batch(squares, blank, seed=k)
    want = oracle.count_many(N, batch)
    assert (want == 0).any() and (want > 0).any()
    got, st = gpu_counts(dls, N, 0, batch, launch=LAUNCHES[li])
    assert st == 0
    assert np.array_equal(got, want), (k, LAUNCHES[li])
