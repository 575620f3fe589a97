"""Host-side logic of the library (no GPU needed): fill order, workunit
split, hourglass canonicalisation and the exported C ABI, each checked
against the oracle or against values the paper prints."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from tests import golden_io

from tests.needs_lib import load as _load_dls  # noqa: E402
dls = _load_dls()
import dls_workloads as workloads  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_are_exported():
    with open(os.path.join(ROOT, "include", "dls.h")) as f:
        text = f.read()
    names = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(dls_[a-z_0-9]+)\s*\(", text, re.M))
    assert {"dls_split", "dls_count", "dls_count_async", "dls_order", "dls_strerror"} <= names
    lib = ctypes.CDLL(dls.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_errors():
    assert "gfx950" in dls.dls_version()
    assert dls.dls_strerror(-1) == "invalid argument"
    with pytest.raises(dls.DLSError):
        dls.dls_order(0)
    with pytest.raises(dls.DLSError):
        dls.dls_split(17, 0, 1)
    with pytest.raises(dls.DLSError):
        dls.dls_split(8, dls.DLS_SYMBREAK, 5)         # depth shorter than the hourglass


# --------------------------------------------------------------------------
# fill order
# --------------------------------------------------------------------------

def test_order_reproduces_fig1():
    assert dls.dls_order(9) == golden_io.fig1_order()


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9, 10, 11])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_order_matches_oracle(n, flags):
    first = oracle.hourglass_cells(n) if flags & 2 else None
    assert dls.dls_order(n, flags) == oracle.fill_order(n, vs=bool(flags & 1), first=first)


def test_order_matches_oracle_random_patterns():
    rng = workloads.SplitMix64(7)
    for trial in range(30):
        n = 5 + rng.below(5)
        vs = bool(rng.below(2))
        p = workloads.random_prefix(n, rng.below(2 * n), vs, rng)
        assigned = (p != 0xFF).astype(np.uint8)
        got = dls.dls_order(n, int(vs), assigned)
        want = oracle.fill_order(n, np.flatnonzero(assigned).tolist(), vs=vs)
        assert got == want, (n, vs)


@pytest.mark.parametrize("n", [4, 5, 7, 8, 9])
@pytest.mark.parametrize("flags", [0, 1, 2])
def test_order_variants_are_valid_orders(n, flags):
    assigned = np.zeros(n * n, dtype=np.uint8)
    assigned[:n] = 1
    paper = dls.dls_order(n, flags, assigned)
    assert dls.dls_order_variant(n, flags, assigned, 0) == paper
    hc = set(oracle.hourglass_cells(n))
    orders = set()
    for v in range(8):
        o = dls.dls_order_variant(n, flags, assigned, v)
        # the same cells as the paper's order, each once
        assert sorted(o) == sorted(paper), v
        if flags & 2:
            # the hourglass comes first whatever the variant
            assert set(o[:len(hc)]) == hc, v
        orders.add(tuple(o))
    if n >= 7:
        assert len(orders) > 1
    for bad in (-1, 8):
        with pytest.raises(dls.DLSError):
            dls.dls_order_variant(n, flags, assigned, bad)


# --------------------------------------------------------------------------
# split
# --------------------------------------------------------------------------

def _oracle_split(n, flags, depth, base=None):
    base = oracle.identity_prefix(n) if base is None else base
    assigned = np.flatnonzero(base != 0xFF).tolist()
    vs = bool(flags & 1)
    order = oracle.fill_order(n, assigned, vs=vs)
    cells = []
    for c in order[:depth]:
        cells.append(c)
        m = (c // n) * n + (n - 1 - c % n)
        if vs and m != c:
            cells.append(m)       # the oracle checks vertical symmetry on the pair
    return oracle.assignments(n, base, cells, vs=vs)


@pytest.mark.parametrize("n,flags,depth", [(5, 0, 6), (6, 0, 8), (7, 0, 11), (7, 0, 14),
                                           (6, 1, 6), (8, 1, 8)])
def test_split_equals_oracle_assignments(n, flags, depth):
    pre, mult = dls.dls_split(n, flags, depth)
    want = _oracle_split(n, flags, depth)
    assert np.array_equal(pre, want)                 # same prefixes, same order
    assert np.all(mult == 1)


def test_split_order9_decomposition():
    # the Sec. 5.2 decomposition (first 10 cells of the Fig. 1 order); the
    # reproducible size, see test_oracle.test_order9_decomposition_size
    pre, _ = dls.dls_split(9, 0, 10)
    assert pre.shape[0] == 1255884
    assert np.all(pre[:, :9] == np.arange(9))


def test_split_from_and_additivity():
    n = 7
    base = oracle.identity_prefix(n)
    base[8] = 2                                       # (1,1) = 2
    kids = dls.dls_split_from(n, 0, base, 5)
    assigned = np.flatnonzero(base != 0xFF).tolist()
    order = oracle.fill_order(n, assigned)
    assert np.array_equal(kids, oracle.assignments(n, base, order[:5]))
    assert int(oracle.count_many(n, kids).sum()) == oracle.count(n, base)


def test_split_from_vs_pairs():
    n = 6
    base = oracle.identity_prefix(n)
    base[n + 1] = 3                                   # (1,1)=3 implies (1,4)=2
    kids = dls.dls_split_from(n, dls.DLS_VSYM, base, 3)
    assert np.all(kids[:, n + 4] == 2)
    bad = base.copy()
    bad[n + 4] = 1                                    # contradicts the mirror of (1,1)
    assert dls.dls_split_from(n, dls.DLS_VSYM, bad, 3).shape[0] == 0


def test_split_sample_positions():
    n, depth = 8, 14
    full, _ = dls.dls_split(n, 0, depth)
    idx = workloads.sample_positions(full.shape[0], 300, seed=3)
    got, total = dls.dls_split_sample(n, 0, depth, idx)
    assert total == full.shape[0]
    assert np.array_equal(got, full[idx])
    with pytest.raises(dls.DLSError):
        dls.dls_split_sample(n, 0, depth, [total])


# --------------------------------------------------------------------------
# symmetry breaking
# --------------------------------------------------------------------------

def test_group_order():
    for n in range(4, 12):
        assert dls.dls_group_order(n) == len(oracle.hourglass_group(n)[0])


@pytest.mark.parametrize("n", [5, 6, 7])
def test_canonical_hourglasses_match_oracle(n):
    hc_depth = len([c for c in dls.dls_order(n, dls.DLS_SYMBREAK)
                    if c in set(oracle.hourglass_cells(n))])
    pre, mult = dls.dls_split(n, dls.DLS_SYMBREAK, hc_depth)
    _, reps, omult = oracle.hourglass_classes(n)
    order = np.lexsort(pre.T[::-1])
    assert np.array_equal(pre[order], reps)
    assert np.array_equal(mult[order], omult)


def test_canonical_hourglasses_order8_pins():
    pins = golden_io.keyed("hourglass_n8.txt")
    pre, mult = dls.dls_split(8, dls.DLS_SYMBREAK, 20)
    assert pre.shape[0] == pins["classes"]
    assert int(mult.astype(np.int64).sum()) == pins["hourglasses"]
    assert int(mult.max()) == pins["max_class"]


@pytest.mark.slow
def test_canonical_hourglasses_order8_equal_oracle():
    pre, mult = dls.dls_split(8, dls.DLS_SYMBREAK, 20)
    _, reps, omult = oracle.hourglass_classes(8)
    order = np.lexsort(pre.T[::-1])
    assert np.array_equal(pre[order], reps)
    assert np.array_equal(mult[order], omult)


def _vs_hourglass_depth(n):
    o = dls.dls_order(n, dls.DLS_VSYM | dls.DLS_SYMBREAK)
    hc = set(oracle.hourglass_cells(n))
    return len([c for c in o if c in hc or (c // n) * n + (n - 1 - c % n) in hc])


@pytest.mark.parametrize("n", [6, 8, 10])
def test_vs_canonical_hourglasses_equal_oracle(n):
    # vertical symmetry with symmetry breaking (Sec. 5.4): the library's
    # product-of-tables group against the oracle's generator closure
    pre, mult = dls.dls_split(n, dls.DLS_VSYM | dls.DLS_SYMBREAK, _vs_hourglass_depth(n))
    nh, reps, omult = oracle.hourglass_classes(n, vs=True)
    order = np.lexsort(pre.T[::-1])
    assert np.array_equal(pre[order], reps)
    assert np.array_equal(mult[order], omult)
    assert int(mult.astype(np.int64).sum()) == nh
    if n == 10:
        # the vertical mirror acts trivially on VS squares: classes of at
        # most 2^5 * 4! = 768 (Sec. 5.4)
        assert int(mult.max()) == 768


def test_canon_single_designs_match_oracle():
    rng = np.random.default_rng(11)
    for n in (6, 7, 8):
        hc = oracle.hourglass_cells(n)
        hs = oracle.assignments(n, oracle.identity_prefix(n), hc[n:] if False else
                                [c for c in hc if c >= n]) if n < 8 else None
        if hs is None:
            pre, _ = dls.dls_split(8, dls.DLS_SYMBREAK, 20)
            p, _ = oracle.hourglass_group(8)
            hs = np.array([oracle.apply(8, int(g), pre[int(k)])
                           for k, g in zip(rng.integers(0, len(pre), 60),
                                           rng.integers(0, len(p), 60))])
        for h in hs[rng.choice(len(hs), size=min(60, len(hs)), replace=False)]:
            assert dls.dls_canon(n, h) == oracle.canon(n, h)


def test_symbreak_split_row1_matches_oracle_order7():
    # hourglass + the next row, as in the order-8 workload, on order 7
    n = 7
    o = dls.dls_order(n, dls.DLS_SYMBREAK)
    hset = set(oracle.hourglass_cells(n))
    hl = len([c for c in o if c in hset])
    depth = hl + (n - 2)
    pre, mult = dls.dls_split(n, dls.DLS_SYMBREAK, depth)
    _, reps, omult = oracle.hourglass_classes(n)
    rows, mults = [], []
    for h, m in zip(reps, omult):
        ext = oracle.assignments(n, h, o[hl:depth])
        rows.append(ext)
        mults.append(np.full(len(ext), m, dtype=np.uint32))
    want = np.concatenate(rows)
    wmult = np.concatenate(mults)
    a = np.lexsort(pre.T[::-1])
    b = np.lexsort(want.T[::-1])
    assert np.array_equal(pre[a], want[b])
    assert np.array_equal(mult[a], wmult[b])


# --------------------------------------------------------------------------
# the input generator
# --------------------------------------------------------------------------

def test_splitmix64_reference_values():
    # published SplitMix64 outputs for seed 0 (Steele, Lea, Flood 2014;
    # the Java SplittableRandom/xoshiro seeding reference)
    r = workloads.SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F]


def test_random_prefixes_are_consistent():
    rng = workloads.SplitMix64(5)
    for _ in range(40):
        n = 6 + rng.below(4)
        vs = bool(rng.below(2))
        p = workloads.random_prefix(n, n + rng.below(2 * n), vs, rng)
        assert oracle.count_assignments(n, p, []) == 1      # locally consistent
        if vs and n % 2 == 0:
            a = p.reshape(n, n).astype(int)
            for i in range(n):
                for j in range(n):
                    if a[i, j] != 255:
                        assert a[i, n - 1 - j] == n - 1 - a[i, j]


def test_single_hip_runtime_in_process():
    # the binding must bind libdls.so to the HIP runtime torch already loaded
    with open("/proc/self/maps") as f:
        libs = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(libs) <= 1, libs


def test_cell_list_errors_before_the_device():
    # a bad cell list is rejected without touching the GPU
    n = 6
    base = oracle.identity_prefix(n)[None]
    for cells, flags in (([0], 0),            # assigned in the prefix
                         ([7, 7], 0),         # repeated
                         ([n * n], 0),        # out of range
                         ([n + n - 1], 1)):   # right half with vertical symmetry
        with pytest.raises(dls.DLSError) as ei:
            dls.dls_count_cells(n, flags, cells, base)
        assert ei.value.code == -1, cells


def _python_cost(n, prefix, order):
    """Entries into levels below the first and squares reached, by plain
    recursion over sets (independent of the library's bitmask code)."""
    sq = [None if v == 0xFF else int(v) for v in prefix]

    def ok(c, v):
        i, j = divmod(c, n)
        for t in range(n):
            if sq[i * n + t] == v or sq[t * n + j] == v:
                return False
        if i == j and any(sq[t * n + t] == v for t in range(n)):
            return False
        if i + j == n - 1 and any(sq[t * n + n - 1 - t] == v for t in range(n)):
            return False
        return True

    steps = leaves = 0

    def rec(k):
        nonlocal steps, leaves
        c = order[k]
        vals = [v for v in range(n) if ok(c, v)]
        if k + 1 == len(order):
            leaves += len(vals)
            return
        for v in vals:
            sq[c] = v
            steps += 1
            rec(k + 1)
            sq[c] = None

    rec(0)
    return steps, leaves


@pytest.mark.parametrize("n", [4, 5, 6])
def test_order_cost_matches_plain_recursion(n):
    base = oracle.identity_prefix(n)
    rng = workloads.SplitMix64(40 + n)
    empty = list(range(n, n * n))
    for trial in range(3):
        order = empty[:]
        for t in range(len(order) - 1, 0, -1):          # Fisher-Yates with the seeded stream
            u = rng.below(t + 1)
            order[t], order[u] = order[u], order[t]
        cut = order[: {4: len(order), 5: 12, 6: 10}[n]]
        steps, leaves = dls.dls_order_cost(n, 0, cut, base[None])
        assert (steps, leaves) == _python_cost(n, base, cut), (n, trial)
    # a full order reaches every square, whatever the order
    st, lv = dls.dls_order_cost(n, 0, dls.dls_order(n), base[None])
    assert lv == oracle.count(n, base)


def test_order_cost_rejects_assigned_cells():
    base = oracle.identity_prefix(6)
    with pytest.raises(dls.DLSError):
        dls.dls_order_cost(6, 0, [0, 7], base[None])


# --------------------------------------------------------------------------
# breadth-first split to a target size (the serving split, Sec. 5.2)
# --------------------------------------------------------------------------

def _oracle_cells(n, vs, order, d):
    cells = []
    for c in order[:d]:
        cells.append(c)
        m = (c // n) * n + (n - 1 - c % n)
        if vs and m != c:
            cells.append(m)
    return cells


@pytest.mark.parametrize("n,vs", [(5, False), (6, False), (7, False), (8, False), (6, True), (8, True)])
def test_split_target_equals_the_oracle_workunits(n, vs):
    rng = workloads.SplitMix64(300 + n + vs)
    for trial in range(6):
        base = workloads.random_prefix(n, rng.below(n + 1), vs, rng)
        target = 1 + rng.below(400)
        got = dls.dls_split_target(n, int(vs), base, target, 24)
        order = oracle.fill_order(n, np.flatnonzero(base != 0xFF).tolist(), vs=vs)
        maxd = min(24, max(0, len(order) - 2))
        # the smallest depth that reaches the target (or the deepest allowed)
        for d in range(maxd + 1):
            want = oracle.assignments(n, base, _oracle_cells(n, vs, order, d), vs=vs)
            if len(want) >= target or d == maxd or len(want) == 0:
                break
        if len(want) == 0:
            assert len(got) == 0
            continue
        a = {bytes(r) for r in got}
        b = {bytes(r) for r in want}
        assert len(a) == len(got) and a == b, (n, vs, trial, d, len(got), len(want))


def test_split_target_counts_sum_to_the_base():
    # Sec. 5.2: the workunits' counts add up to the count of the prefix
    n = 6
    rng = workloads.SplitMix64(17)
    for vs in (False, True):
        base = workloads.random_prefix(n, 3, vs, rng)
        units = dls.dls_split_target(n, int(vs), base, 50, 24)
        assert int(oracle.count_many(n, units, vs=vs).sum()) == oracle.count(n, base, vs=vs)
