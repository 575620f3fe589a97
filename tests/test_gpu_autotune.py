"""GPU test of the autotuner: every candidate launch must produce the same
counts (the tuner checks a digest of them and refuses a difference), the
fastest is kept, and the plain-kernel reference is optional.  Nothing is
written to the tuning cache."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_tune_small_space_without_saving():
    from paper_1709_02599_amd import autotune
    pre, _ = dls.dls_split(7, 0, 11)
    space = {"order_variant": (0, 5), "refill_every": (16, 64)}
    r = autotune.tune(7, 0, pre, "test-order7", space=space, default={"order_variant": 0, "refill_every": 16},
                      reps=1, save=False, verbose=False)
    assert r["candidates"] == 4 and r["prefixes"] == len(pre)
    times = [row["ms"] for row in r["table"]]
    assert times == sorted(times) and r["best"] == r["table"][0]
    assert r["default"]["order_variant"] == 0 and r["default"]["refill_every"] == 16
    assert r["plain_ms"] is not None and r["plain_ms"] > 0
    r2 = autotune.tune(7, 0, pre, "test-order7", space={"order_variant": (1,)}, reps=1, save=False,
                       verbose=False, plain=False)
    assert r2["plain_ms"] is None and r2["candidates"] == 1
    assert autotune.best(7, 0, "test-order7") is None   # nothing was saved
