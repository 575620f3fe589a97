"""Resumable chunked full counts: chunks of an interleaved split, resumed
after an interruption and merged, give the oracle's total."""
import json

import pytest

import oracle

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_chunks_resume_and_merge(tmp_path):
    from paper_1709_02599_amd import fullcount
    n = 7
    o = dls.dls_order(n, dls.DLS_SYMBREAK)
    hset = set(oracle.hourglass_cells(n))
    depth = len([c for c in o if c in hset]) + 2
    out = str(tmp_path)
    # chunk 1 is interrupted after one of its three batches, then resumed
    fullcount.run_chunk(n, dls.DLS_SYMBREAK, depth, 1, 3, out, batches=3, log=lambda s: None, stop_after=1)
    with open(fullcount._path(out, 1, 3)) as f:
        assert json.load(f)["done_batches"] == 1
    assert not fullcount.merge(out)["complete"]
    for c in range(3):
        fullcount.run_chunk(n, dls.DLS_SYMBREAK, depth, c, 3, out, batches=3, log=lambda s: None)
    m = fullcount.merge(out)
    assert m["complete"] and m["missing_chunks"] == []
    assert m["weighted_sum"] == oracle.count(n, oracle.identity_prefix(n))
