"""Hourglass designs and their canonical forms on the GPU (Alg. 5) against
the host's split with symmetry breaking and the oracle's classes."""
import numpy as np
import pytest

import oracle
from tests import golden_io
from tests.gpu_helpers import gpu_counts, weighted_total

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _hl(n):
    o = dls.dls_order(n, dls.DLS_SYMBREAK)
    hset = set(oracle.hourglass_cells(n))
    return len([c for c in o if c in hset])


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_classes_equal_oracle(n):
    pre, mult = dls.hourglass_classes_gpu(n)
    nh, reps, omult = oracle.hourglass_classes(n)
    assert np.array_equal(pre, reps) and np.array_equal(mult, omult)
    assert int(mult.astype(np.int64).sum()) == nh


def test_classes_order8_pins_and_host():
    pre, mult = dls.hourglass_classes_gpu(8)
    pins = golden_io.keyed("hourglass_n8.txt")
    assert len(pre) == pins["classes"]
    assert int(mult.astype(np.int64).sum()) == pins["hourglasses"]
    assert int(mult.max()) == pins["max_class"]
    hpre, hmult = dls.dls_split(8, dls.DLS_SYMBREAK, _hl(8))
    order = np.lexsort(hpre.T[::-1])
    assert np.array_equal(pre, hpre[order]) and np.array_equal(mult, hmult[order])


def test_symmetry_broken_count_from_gpu_classes():
    # classes from the GPU, completions counted on the GPU: sum(mult * count)
    # is the number of order-7 DLS with the first row fixed
    n = 7
    pre, mult = dls.hourglass_classes_gpu(n)
    c, st = gpu_counts(dls, n, 0, pre)
    assert st == 0
    assert weighted_total(c, mult) == oracle.count(n, oracle.identity_prefix(n))
