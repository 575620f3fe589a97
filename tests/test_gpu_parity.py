"""GPU parity: the HIP kernels, called through the C ABI, against the CPU
oracle, count for count (exact integers: tolerance 0).  Needs an MI355X.

The oracle never sees an input produced by the library: where a workload is a
split, the oracle builds the same prefix list itself and the two lists are
compared first; counts are then compared element by element."""
import numpy as np
import pytest

import oracle
from tests import golden_io
from tests.gpu_helpers import gpu_counts, weighted_total

pytestmark = pytest.mark.gpu

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()
import dls_workloads as workloads  # noqa: E402

E = 0xFF
KERNELS = [False, True]          # persistent, plain


def _oracle_split(n, vs, depth, first=None, base=None):
    base = oracle.identity_prefix(n) if base is None else base
    order = oracle.fill_order(n, np.flatnonzero(base != E).tolist(), vs=vs, first=first)
    cells = []
    for c in order[:depth]:
        cells.append(c)
        m = (c // n) * n + (n - 1 - c % n)
        if vs and m != c:
            cells.append(m)
    return oracle.assignments(n, base, cells, vs=vs)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[gpu] device:", torch.cuda.get_device_name(0), flush=True)


# --------------------------------------------------------------------------
# single prefixes, every small order
# --------------------------------------------------------------------------

@pytest.mark.parametrize("plain", KERNELS)
def test_order6_single_prefix(plain):
    # one launch, one prefix: row 0 = 0..5
    c, st = gpu_counts(dls, 6, 0, oracle.identity_prefix(6)[None], plain=plain)
    want = oracle.count(6, oracle.identity_prefix(6))
    assert st == 0 and int(c[0]) == want
    assert oracle.total_from_fixed(6, int(c[0])) == oracle.count(6, np.full(36, E, np.uint8))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
@pytest.mark.parametrize("vs", [False, True])
@pytest.mark.parametrize("plain", KERNELS)
def test_small_orders(n, vs, plain):
    p = oracle.identity_prefix(n)[None]
    c, st = gpu_counts(dls, n, dls.DLS_VSYM if vs else 0, p, plain=plain)
    assert st == 0 and int(c[0]) == oracle.count(n, p[0], vs=vs)


def test_host_api_mixed_patterns():
    rng = workloads.SplitMix64(99)
    pres = [workloads.random_prefix(7, 4 + rng.below(10), False, rng) for _ in range(40)]
    pres = np.stack(pres)
    for flags in (0, dls.DLS_PLAIN):
        got = dls.dls_count(7, flags, pres)
        assert np.array_equal(got, oracle.count_many(7, pres))


# --------------------------------------------------------------------------
# order 7, split on the diagonals (uneven subtrees)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("plain", KERNELS)
@pytest.mark.parametrize("block", [64, 256, 1024])
def test_order7_diagonal_split(plain, block):
    pre, _ = dls.dls_split(7, 0, 11)
    opre = _oracle_split(7, False, 11)
    assert np.array_equal(pre, opre)
    c, st = gpu_counts(dls, 7, 0, pre, plain=plain, launch={"block": block})
    assert st == 0
    assert np.array_equal(c, oracle.count_many(7, opre))
    assert int(c.sum()) == oracle.count(7, oracle.identity_prefix(7))


def test_persistent_refill_and_steal_settings_agree():
    pre, _ = dls.dls_split(7, 0, 8)
    want = oracle.count_many(7, _oracle_split(7, False, 8))
    for launch in ({"refill_every": 1, "steal_depth": 3}, {"refill_every": 64, "steal_depth": 12},
                   {"block": 128, "blocks_per_cu": 1, "refill_every": 8, "steal_depth": 4}):
        c, st = gpu_counts(dls, 7, 0, pre, launch=launch)
        assert st == 0 and np.array_equal(c, want), launch


def test_persistent_single_heavy_prefix_is_shared_out():
    # one prefix for the whole GPU: only donation spreads the work
    for n in (7, 8):
        p = oracle.identity_prefix(n)
        if n == 8:
            p = _oracle_split(8, False, 14)[1000]
        c, st = gpu_counts(dls, n, 0, p[None], launch={"steal_depth": 4})
        assert st == 0 and int(c[0]) == oracle.count(n, p)


# --------------------------------------------------------------------------
# breadth-first expansion of small batches before the persistent kernel
# --------------------------------------------------------------------------

@pytest.mark.parametrize("target", [-1, 1, 7, 100, 5000, 0])   # off, tiny, ..., default
def test_expansion_targets_order7(target):
    pre, _ = dls.dls_split(7, 0, 11)
    opre = _oracle_split(7, False, 11)
    want = oracle.count_many(7, opre)
    c, st = gpu_counts(dls, 7, 0, pre, launch={"expand_target": target})
    assert st == 0 and np.array_equal(c, want), target


@pytest.mark.parametrize("n,vs", [(4, False), (5, False), (6, False), (7, False), (6, True), (8, True)])
@pytest.mark.parametrize("target", [3, 1000, 0])
def test_expansion_single_prefix(n, vs, target):
    # one prefix: every task after the passes shares its count slot
    p = oracle.identity_prefix(n)
    c, st = gpu_counts(dls, n, dls.DLS_VSYM if vs else 0, p[None], launch={"expand_target": target})
    assert st == 0 and int(c[0]) == oracle.count(n, p, vs=vs)


def test_expansion_mixed_dead_and_live_prefixes():
    # every third prefix made inconsistent (a value repeated on the main
    # diagonal), the others live: dead tasks drop out of the passes
    pre, _ = dls.dls_split(7, 0, 11)
    pre = pre.copy()
    pre[::3, 2 * 7 + 2] = pre[::3, 1 * 7 + 1]
    want = oracle.count_many(7, pre)
    assert np.all(want[::3] == 0)
    for target in (2, 50, 0):
        c, st = gpu_counts(dls, 7, 0, pre, launch={"expand_target": target})
        assert st == 0 and np.array_equal(c, want), target


def test_expansion_reused_buffers_start_clean():
    # the per-task count slots of one launch must not leak into the next on
    # the same stream: alternate two batches several times
    a, _ = dls.dls_split(7, 0, 8)
    b, _ = dls.dls_split(7, 0, 11)
    wa = oracle.count_many(7, _oracle_split(7, False, 8))
    wb = oracle.count_many(7, _oracle_split(7, False, 11))
    for rep in range(3):
        for pre, want in ((a, wa), (b, wb)):
            c, st = gpu_counts(dls, 7, 0, pre)
            assert st == 0 and np.array_equal(c, want), (rep, len(pre))


def test_expansion_capacity_bounds_a_pass():
    # a target whose 4x capacity is below the next level's candidate count:
    # the passes stop early and the search finishes the rest
    pre, _ = dls.dls_split(7, 0, 8)
    want = oracle.count_many(7, _oracle_split(7, False, 8))
    for target in (len(pre) + 1, 2 * len(pre), 3 * len(pre)):
        c, st = gpu_counts(dls, 7, 0, pre, launch={"expand_target": target})
        assert st == 0 and np.array_equal(c, want), target


# --------------------------------------------------------------------------
# order 8 with symmetry breaking: canonical hourglasses + row 1
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def order8_symbreak():
    n = 8
    pre, mult = dls.dls_split(n, dls.DLS_SYMBREAK, 26)
    # the oracle's own list: its canonical hourglasses, each extended by the
    # next six cells of its own fill order (row 1)
    hc = oracle.hourglass_cells(n)
    order = oracle.fill_order(n, first=hc)
    hl = len([c for c in order if c in set(hc)])
    _, reps, rmult = oracle.hourglass_classes(n)
    rows, mults = [], []
    for h, m in zip(reps, rmult):
        ext = oracle.assignments(n, h, order[hl:hl + 6])
        rows.append(ext)
        mults.append(np.full(len(ext), m, np.uint32))
    opre = np.concatenate(rows)
    omult = np.concatenate(mults)
    a = np.lexsort(pre.T[::-1])
    b = np.lexsort(opre.T[::-1])
    # every workunit counted by the oracle (seconds on the host's threads)
    ocounts = oracle.count_many(n, opre)
    return pre, mult, opre, omult, a, b, ocounts


def test_order8_symbreak_prefix_lists_agree(order8_symbreak):
    pre, mult, opre, omult, a, b, _ = order8_symbreak
    assert pre.shape == opre.shape
    assert np.array_equal(pre[a], opre[b])
    assert np.array_equal(mult[a], omult[b])


@pytest.mark.parametrize("plain", KERNELS)
def test_order8_symbreak_counts(order8_symbreak, plain):
    pre, mult, opre, omult, a, b, ocounts = order8_symbreak
    c, st = gpu_counts(dls, 8, 0, pre, plain=plain)
    assert st == 0
    # Corollary 1: sum of class power x count is the fixed-first-row total
    assert weighted_total(c, mult) == golden_io.counts()[(8, "fixed")]
    # all 2 819 311 workunits, element by element against the oracle
    assert np.array_equal(c[a], ocounts[b])


def test_order8_symbreak_tuned_launch_counts(order8_symbreak):
    # the launch the benchmark times (fill-order variant 5, VGPR masks,
    # 8 workgroups of 512 per CU, refill every 64 steps when two lanes are
    # idle, chunks >= 64, the workgroup pool of the tail on)
    pre, mult, opre, omult, a, b, ocounts = order8_symbreak
    launch = {"block": 512, "blocks_per_cu": 8, "refill_every": 64, "order_variant": 5,
              "chunk_min": 64, "lds_masks": -1, "refill_min": 2}
    c, st = gpu_counts(dls, 8, 0, pre, launch=launch)
    assert st == 0
    assert np.array_equal(c[a], ocounts[b])


@pytest.mark.parametrize("block", [64, 128, 1024])
@pytest.mark.parametrize("wg_pool", [0, -1, 3])
def test_order8_symbreak_workgroup_pool(order8_symbreak, block, wg_pool):
    # the tail's workgroup pool on (as many records as fit, or only 3),
    # and off, for 1, 2 and 16 waves per workgroup (the stack slots are
    # dealt out per bank only when the waves fill the words: not at 64 or
    # 128 lanes with byte slots); every count against the oracle
    pre, mult, opre, omult, a, b, ocounts = order8_symbreak
    launch = {"block": block, "blocks_per_cu": max(1, 2048 // block), "refill_every": 32,
              "order_variant": 5, "lds_masks": -1, "wg_pool": wg_pool}
    c, st = gpu_counts(dls, 8, 0, pre, launch=launch)
    assert st == 0
    assert np.array_equal(c[a], ocounts[b])


def test_order8_symbreak_kernels_agree_everywhere(order8_symbreak):
    pre = order8_symbreak[0]
    c1, s1 = gpu_counts(dls, 8, 0, pre)
    c2, s2 = gpu_counts(dls, 8, 0, pre, plain=True)
    c3, s3 = gpu_counts(dls, 8, 0, pre, launch={"block": 512, "refill_every": 16})
    assert s1 == s2 == s3 == 0
    assert np.array_equal(c1, c2) and np.array_equal(c1, c3)


# --------------------------------------------------------------------------
# vertical symmetry
# --------------------------------------------------------------------------

@pytest.mark.parametrize("plain", KERNELS)
def test_vs_order8_full_count(plain):
    n = 8
    pre, _ = dls.dls_split(n, dls.DLS_VSYM, 12)
    opre = _oracle_split(n, True, 12)
    assert np.array_equal(pre, opre)
    c, st = gpu_counts(dls, n, dls.DLS_VSYM, pre, plain=plain)
    assert st == 0
    assert int(c.sum()) == oracle.count(n, oracle.identity_prefix(n), vs=True)
    # all 114 960 workunits, element by element
    assert np.array_equal(c, oracle.count_many(n, opre, vs=True))


def test_order8_full_count_without_symmetry_breaking():
    # the sustained workload: the 14 diagonal cells split on the host
    # (547 896 workunits), every one of the 7 447 587 840 squares with the
    # first row fixed (Sec. 5.1); 2 000 seeded workunits element by element
    n = 8
    pre, _ = dls.dls_split(n, 0, 14)
    assert len(pre) == 547_896
    opre = _oracle_split(n, False, 14)
    assert np.array_equal(pre, opre)
    pos = workloads.sample_positions(len(pre), 2000, seed=14)
    want = oracle.count_many(n, opre[pos])
    for launch in (None, {"order_variant": 1}):
        c, st = gpu_counts(dls, n, 0, pre, launch=launch)
        assert st == 0
        assert int(c.sum()) == golden_io.counts()[(8, "fixed")]
        assert np.array_equal(c[pos], want), launch


def test_vs_odd_order_is_zero():
    p = np.stack([oracle.identity_prefix(7)] * 3)
    c, st = gpu_counts(dls, 7, dls.DLS_VSYM, p)
    assert st == 0 and np.all(c == 0)


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("plain", KERNELS)
def test_complete_and_nearly_complete_squares(plain):
    n = 5
    full = oracle.assignments(n, oracle.identity_prefix(n), list(range(n, n * n)))
    c, st = gpu_counts(dls, n, 0, full, plain=plain)
    assert st == 0 and np.all(c == 1)
    bad = full.copy()
    bad[:, [n, n + 1]] = bad[:, [n + 1, n]]
    c, st = gpu_counts(dls, n, 0, bad, plain=plain)
    assert st == 0 and np.all(c == 0)
    one = full.copy()
    one[:, n * n - 1] = E                         # a single empty cell
    c, st = gpu_counts(dls, n, 0, one, plain=plain)
    assert st == 0 and np.all(c == 1)


@pytest.mark.parametrize("plain", KERNELS)
def test_inconsistent_prefixes_and_ragged_tail(plain):
    pre, _ = dls.dls_split(7, 0, 6)
    pre = pre[:1001].copy()                       # not a multiple of any block size
    pre[::7, 8] = pre[::7, 0]                     # (1,1) = (0,0): main-diagonal clash
    c, st = gpu_counts(dls, 7, 0, pre, plain=plain, launch={"block": 128})
    assert st == 0
    assert np.array_equal(c, oracle.count_many(7, pre))
    assert np.all(c[::7] == 0)


@pytest.mark.parametrize("flags", [0, dls.DLS_PLAIN])
def test_count_async_six_arguments(flags):
    # the scope-table form: device prefixes and counts on a stream, pattern
    # read from prefix 0, status kept by the library per stream
    import torch
    n = 7
    pre, _ = dls.dls_split(n, 0, 11)
    want = oracle.count_many(n, oracle.assignments(n, oracle.identity_prefix(n), oracle.fill_order(n)[:11]))
    st = torch.cuda.Stream()
    d_pre = torch.from_numpy(pre).cuda()
    d_cnt = torch.full((len(pre),), -1, dtype=torch.int64, device="cuda")
    dls.dls_count_async(n, flags, d_pre, len(pre), d_cnt, st)
    assert dls.dls_stream_status(st) == 0
    assert np.array_equal(d_cnt.cpu().numpy().view(np.uint64), want)
    # a prefix with another pattern counts 0 and is reported on the stream
    bad = pre[:16].copy()
    free = int(np.flatnonzero(pre[0] == E)[-1])    # a cell no prefix assigns
    bad[5, free] = 3
    d_bad = torch.from_numpy(bad).cuda()
    d_c2 = torch.zeros(16, dtype=torch.int64, device="cuda")
    dls.dls_count_async(n, flags, d_bad, 16, d_c2, st)
    assert dls.dls_stream_status(st) & 1
    got = d_c2.cpu().numpy().view(np.uint64)
    assert got[5] == 0 and np.array_equal(np.delete(got, 5), np.delete(want[:16], 5))
    assert dls.dls_stream_status(st) == 0          # read clears the word


def test_count_async_vs_six_arguments():
    import torch
    pre, _ = dls.dls_split(8, dls.DLS_VSYM, 10)
    sel = pre[workloads.sample_positions(len(pre), 200, seed=11)]
    d_pre = torch.from_numpy(sel).cuda()
    d_cnt = torch.zeros(len(sel), dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    dls.dls_count_async(8, dls.DLS_VSYM, d_pre, len(sel), d_cnt, s)
    assert dls.dls_stream_status(s) == 0
    assert np.array_equal(d_cnt.cpu().numpy().view(np.uint64), oracle.count_many(8, sel, vs=True))


def test_pattern_mismatch_flagged():
    pre, _ = dls.dls_split(6, 0, 4)
    pre = pre[:10].copy()
    pre[3, 35] = 0                                # an extra assigned cell
    c, st = gpu_counts(dls, 6, 0, pre)
    assert st & 1
    assert c[3] == 0


def test_empty_batch():
    import torch
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    dls.dls_count_async(6, 0, d, 0, d)            # nothing to do
    torch.cuda.synchronize()
    assert dls.dls_count(6, 0, np.zeros((0, 36), np.uint8)).shape == (0,)


def test_vs_order10_sampled_prefixes():
    # 4096 seeded positions of the VS order-10 split at depth 17 (Sec. 5.4):
    # the library's sampled prefixes equal the oracle's, every count equals
    # the oracle's, and the estimate total x mean matches the paper's count
    total, cells, pos, opre, ocounts = golden_io.vs10_sample()
    pre, ptotal = dls.dls_split_sample(10, dls.DLS_VSYM, 17, pos)
    assert ptotal == total
    assert np.array_equal(pre, opre)
    c, st = gpu_counts(dls, 10, dls.DLS_VSYM, pre)
    assert st == 0
    assert np.array_equal(c, ocounts)
    x = c.astype(np.float64)
    est = total * x.mean()
    se = total * x.std(ddof=1) / np.sqrt(len(x))
    paper = golden_io.counts()[(10, "vs_fixed")]
    assert abs(est - paper) < 3 * se, (est, paper, se)


def _oracle_vs_symbreak_split(n, extra):
    """The oracle's own workunits: its canonical VS hourglasses, each extended
    by all fillings of the next `extra` left-half cells of its own order."""
    hc = oracle.hourglass_cells(n)
    order = oracle.fill_order(n, first=hc, vs=True)
    hset = set(hc)
    hl = len([c for c in order if c in hset or (c // n) * n + (n - 1 - c % n) in hset])
    cells = []
    for c in order[hl:hl + extra]:
        cells.append(c)
        m = (c // n) * n + (n - 1 - c % n)
        if m != c:
            cells.append(m)
    _, reps, rmult = oracle.hourglass_classes(n, vs=True)
    rows, mults = [], []
    for h, m in zip(reps, rmult):
        ext = oracle.assignments(n, h, cells, vs=True)
        rows.append(ext)
        mults.append(np.full(len(ext), m, np.uint32))
    return hl, np.concatenate(rows), np.concatenate(mults)


def test_vs_order8_symmetry_broken_total():
    n = 8
    hl, opre, omult = _oracle_vs_symbreak_split(n, 2)
    pre, mult = dls.dls_split(n, dls.DLS_VSYM | dls.DLS_SYMBREAK, hl + 2)
    a, b = np.lexsort(pre.T[::-1]), np.lexsort(opre.T[::-1])
    assert np.array_equal(pre[a], opre[b]) and np.array_equal(mult[a], omult[b])
    c, st = gpu_counts(dls, n, dls.DLS_VSYM, pre)
    assert st == 0
    assert np.array_equal(c[a], oracle.count_many(n, opre[b], vs=True))
    assert weighted_total(c, mult) == oracle.count(n, oracle.identity_prefix(n), vs=True)


def test_vs_order10_full_count_with_symmetry_breaking():
    # Sec. 5.4: all vertically symmetric DLS of order 10 with the first row
    # fixed, through the 9 508 canonical VS hourglasses (classes of up to 768)
    # extended by two more cell pairs: 165 316 workunits, about 1.1e11 squares
    n = 10
    hl, opre, omult = _oracle_vs_symbreak_split(n, 2)
    pre, mult = dls.dls_split(n, dls.DLS_VSYM | dls.DLS_SYMBREAK, hl + 2)
    a, b = np.lexsort(pre.T[::-1]), np.lexsort(opre.T[::-1])
    assert np.array_equal(pre[a], opre[b]) and np.array_equal(mult[a], omult[b])
    c, st = gpu_counts(dls, n, dls.DLS_VSYM, pre)
    assert st == 0
    assert weighted_total(c, mult) == golden_io.counts()[(10, "vs_fixed")]
    # element-wise parity on seeded positions the oracle counts one by one
    pos = workloads.sample_positions(len(pre), 24, seed=1054)
    assert np.array_equal(c[a][pos], oracle.count_many(n, opre[b][pos], vs=True))


# --------------------------------------------------------------------------
# line masks in LDS (LdsLane) instead of VGPRs
# --------------------------------------------------------------------------

LDS_MASKS = {"lds_masks": 1}


@pytest.mark.parametrize("n,vs", [(4, False), (5, False), (6, False), (7, False), (6, True), (8, True)])
def test_lds_masks_single_prefix(n, vs):
    p = oracle.identity_prefix(n)
    for launch in ({**LDS_MASKS, "expand_target": -1}, LDS_MASKS):
        c, st = gpu_counts(dls, n, dls.DLS_VSYM if vs else 0, p[None], launch=launch)
        assert st == 0 and int(c[0]) == oracle.count(n, p, vs=vs), launch


@pytest.mark.parametrize("block", [64, 256, 512])
def test_lds_masks_order7_split_and_donation(block):
    pre, _ = dls.dls_split(7, 0, 8)
    want = oracle.count_many(7, _oracle_split(7, False, 8))
    for extra in ({}, {"steal_depth": 4, "expand_target": -1, "refill_every": 4}):
        c, st = gpu_counts(dls, 7, 0, pre, launch={**LDS_MASKS, "block": block, **extra})
        assert st == 0 and np.array_equal(c, want), (block, extra)


def test_lds_masks_order8_symbreak(order8_symbreak):
    pre, mult, opre, omult, a, b, ocounts = order8_symbreak
    c1, s1 = gpu_counts(dls, 8, 0, pre, launch=LDS_MASKS)
    c2, s2 = gpu_counts(dls, 8, 0, pre, launch={**LDS_MASKS, "block": 512, "order_variant": 5})
    assert s1 == s2 == 0
    assert np.array_equal(c1[a], ocounts[b]) and np.array_equal(c2[a], ocounts[b])
    assert weighted_total(c1, mult) == golden_io.counts()[(8, "fixed")]


def test_lds_masks_vs_order10_sample():
    total, cells, pos, opre, ocounts = golden_io.vs10_sample()
    c, st = gpu_counts(dls, 10, dls.DLS_VSYM, opre[:512], launch=LDS_MASKS)
    assert st == 0 and np.array_equal(c, ocounts[:512])


# --------------------------------------------------------------------------
# line masks forced into VGPRs at orders 9 and 10 (two 64-bit words per kind
# of line); orders >= 9 default to the LDS-mask layout
# --------------------------------------------------------------------------

VGPR_MASKS = {"lds_masks": -1}


@pytest.fixture(scope="module")
def order9_deep():
    """256 order-9 prefixes sharing one pattern: the first 28 cells of the
    fill order assigned (14 at spread positions of the oracle's enumeration,
    then the first consistent extension), with their oracle counts."""
    base = oracle.identity_prefix(9)
    order = oracle.fill_order(9, list(range(9)))
    total = oracle.count_assignments(9, base, order[:14])
    p14 = oracle.assignments_at(9, base, order[:14], np.linspace(0, total - 1, 256).astype(np.int64))
    pattern = np.full(81, 0xFF, dtype=np.uint8)
    pattern[list(range(9)) + list(order[:28])] = 0
    pre = []
    for p in p14:
        if oracle.count_assignments(9, p, order[14:28]) == 0:
            continue  # no consistent extension of this one
        e = oracle.assignments_at(9, p, order[14:28], [0])[0]
        assert np.array_equal(e == 0xFF, pattern == 0xFF)
        pre.append(e)
    pre = np.ascontiguousarray(np.array(pre, dtype=np.uint8))
    return pre, oracle.count_many(9, pre)


@pytest.mark.parametrize("extra", [{}, {"expand_target": -1, "steal_depth": 4, "refill_every": 4},
                                   {"block": 64, "blocks_per_cu": 1, "refill_every": 2}])
def test_order9_both_layouts(order9_deep, extra):
    pre, want = order9_deep
    assert len(pre) > 200 and want.sum() > 0
    for layout in (VGPR_MASKS, LDS_MASKS):
        c, st = gpu_counts(dls, 9, 0, pre, launch={**layout, **extra})
        assert st == 0 and np.array_equal(c, want), (layout, extra)


def test_vgpr_masks_vs_order10_sample():
    total, cells, pos, opre, ocounts = golden_io.vs10_sample()
    c, st = gpu_counts(dls, 10, dls.DLS_VSYM, opre[:512], launch=VGPR_MASKS)
    assert st == 0 and np.array_equal(c, ocounts[:512])
