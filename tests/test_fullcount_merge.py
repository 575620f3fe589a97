"""Merging chunk files of a resumable count (host logic only)."""
import json
import os

import pytest

from tests.needs_lib import load as _load_dls

_load_dls()
from paper_1709_02599_amd import fullcount  # noqa: E402


def _write(d, chunk, chunks, ws, done=3, digest="abc", n=9):
    st = {"n": n, "flags": 2, "depth": 22, "chunk": chunk, "chunks": chunks, "workunits": 100,
          "split_digest": digest, "batches": 3, "done_batches": done, "weighted_sum": str(ws),
          "squares": str(ws // 7), "kernel_seconds": 1.5}
    with open(fullcount._path(d, chunk, chunks), "w") as f:
        json.dump(st, f)


def test_merge_sums_complete_chunks(tmp_path):
    d = str(tmp_path)
    big = 5056994653507584
    _write(d, 0, 3, big // 3)
    _write(d, 1, 3, big // 3)
    _write(d, 2, 3, big - 2 * (big // 3))
    m = fullcount.merge(d)
    assert m["complete"] and m["weighted_sum"] == big and m["missing_chunks"] == []


def test_merge_reports_missing_and_unfinished(tmp_path):
    d = str(tmp_path)
    _write(d, 0, 3, 10)
    _write(d, 2, 3, 10, done=1)
    m = fullcount.merge(d)
    assert not m["complete"] and m["missing_chunks"] == [1, 2]


def test_merge_rejects_mixed_splits(tmp_path):
    d = str(tmp_path)
    _write(d, 0, 2, 10)
    _write(d, 1, 2, 10, digest="other")
    with pytest.raises(RuntimeError):
        fullcount.merge(d)


def test_merge_needs_files(tmp_path):
    with pytest.raises(RuntimeError):
        fullcount.merge(os.path.join(str(tmp_path), "none"))


def test_split_cache_round_trip_and_rebuild(tmp_path, monkeypatch):
    import numpy as np
    from paper_1709_02599_amd import DLS_SYMBREAK, dls_split
    cache = str(tmp_path / "split7.npz")
    pre0, mult0 = dls_split(7, DLS_SYMBREAK, 16)
    pre1, mult1 = fullcount.load_split(7, DLS_SYMBREAK, 16, cache)      # computes, writes
    assert os.path.exists(cache)
    def no_split(*args):
        raise AssertionError("split recomputed although cached")
    with monkeypatch.context() as m:
        m.setattr(fullcount, "dls_split", no_split)
        pre2, mult2 = fullcount.load_split(7, DLS_SYMBREAK, 16, cache)  # reads
    for a, b in ((pre0, pre1), (pre0, pre2), (mult0, mult1), (mult0, mult2)):
        assert np.array_equal(a, b)
    # another split's parameters: rebuilt, not reused
    pre3, _ = fullcount.load_split(7, DLS_SYMBREAK, 17, cache)
    assert np.array_equal(pre3, dls_split(7, DLS_SYMBREAK, 17)[0])
    # a tampered cache fails its digest and is rebuilt
    with np.load(cache) as z:
        d = {k: z[k] for k in z.files}
    d["mult"] = d["mult"] + 1
    np.savez(cache, **d)
    pre4, mult4 = fullcount.load_split(7, DLS_SYMBREAK, 17, cache)
    assert np.array_equal(mult4, dls_split(7, DLS_SYMBREAK, 17)[1])
