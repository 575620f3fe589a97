"""Plain CPU oracle for counting diagonal Latin squares -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library under
``paper_1709_02599_amd/`` never imports it, and the two share no code.

What is here (each item follows a passage of Kochemazov, Vatutin, Zaikin,
arXiv:1709.02599):

* ``count`` / ``count_many`` -- the number of completions of a partial square
  into a diagonal Latin square (definition of Sec. 1), by the plain nested-loop
  search of Algorithms 1-2 (Sec. 2.2) in C (``dls_oracle.c``); ``vs=True``
  adds the vertical-symmetry condition of Sec. 5.4 as a checked constraint.
* ``assignments`` -- all consistent assignments of a list of cells, i.e. the
  workunits of Sec. 5.2.
* ``hourglass_group`` / ``canon`` / ``apply`` / ``hourglass_classes`` -- the
  M-transformations of Sec. 4.1 restricted to hourglass designs (Sec. 4.2),
  the canonicity test and class power of Algorithm 5, and Corollary 1.
* ``brute_force_count`` -- a second, unrelated construction (rows as whole
  permutations, Sec. 2.1) used only to pin the oracle on tiny orders.
* ``fill_order`` -- the most-constrained-cell rule and the forced-cell rule of
  Sec. 2.3, written from the text; pinned by Fig. 1.
* ``total_from_fixed`` -- first-row normalisation (Sec. 2.2): totals are the
  fixed-first-row counts times N! (times 2^(N/2) (N/2)! for VS squares).
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

EMPTY = 0xFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dls_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/_build/liboracle.so``."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_count.restype = ctypes.c_int64
    lib.oracle_count.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
    lib.oracle_count_many.restype = ctypes.c_int
    lib.oracle_count_many.argtypes = [ctypes.c_int, ctypes.c_int, u8p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    lib.oracle_assignments.restype = ctypes.c_int64
    lib.oracle_assignments.argtypes = [ctypes.c_int, ctypes.c_int, u8p,
                                       ctypes.POINTER(ctypes.c_int), ctypes.c_int, u8p,
                                       ctypes.c_int64]
    lib.oracle_assignments_at.restype = ctypes.c_int64
    lib.oracle_assignments_at.argtypes = [ctypes.c_int, ctypes.c_int, u8p,
                                          ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, u8p]
    lib.oracle_first.restype = ctypes.c_int
    lib.oracle_first.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, ctypes.c_int64, u8p]
    lib.oracle_hourglass_group.restype = ctypes.c_int
    lib.oracle_hourglass_group.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int8),
                                           ctypes.POINTER(ctypes.c_int8), ctypes.c_int]
    lib.oracle_canon.restype = ctypes.c_int
    lib.oracle_canon.argtypes = [ctypes.c_int, u8p]
    lib.oracle_apply.restype = ctypes.c_int
    lib.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
    lib.oracle_hourglass_classes.restype = ctypes.c_int64
    lib.oracle_hourglass_classes.argtypes = [ctypes.c_int, ctypes.c_int, u8p,
                                             ctypes.POINTER(ctypes.c_uint32), ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
    _lib = lib
    return lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _square(n: int, cells) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(cells, dtype=np.uint8).reshape(n * n))
    return a


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def identity_prefix(n: int) -> np.ndarray:
    """Row 0 = 0..n-1, every other cell empty (the normalisation of Sec. 2.2)."""
    a = np.full(n * n, EMPTY, dtype=np.uint8)
    a[:n] = np.arange(n, dtype=np.uint8)
    return a


# --------------------------------------------------------------------------
# counting
# --------------------------------------------------------------------------

def count(n: int, cells, vs: bool = False) -> int:
    """Exact number of DLS (VS-DLS if ``vs``) of order n agreeing with cells."""
    r = _load().oracle_count(n, int(bool(vs)), _u8(_square(n, cells)))
    if r < 0:
        raise ValueError("invalid oracle input")
    return int(r)


def count_many(n: int, prefixes: np.ndarray, vs: bool = False,
               threads: Optional[int] = None) -> np.ndarray:
    """Per-prefix exact counts, prefixes shaped [P, n*n] uint8."""
    p = np.ascontiguousarray(np.asarray(prefixes, dtype=np.uint8).reshape(-1, n * n))
    out = np.zeros(p.shape[0], dtype=np.uint64)
    if p.shape[0] == 0:
        return out
    r = _load().oracle_count_many(n, int(bool(vs)), _u8(p), p.shape[0],
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  threads or default_threads())
    if r != 0:
        raise ValueError("invalid oracle input")
    return out


def first_completion(n: int, cells, value_order=None, vs: bool = False,
                     node_limit: int = 10_000_000) -> Optional[np.ndarray]:
    """One square agreeing with ``cells`` (the same search as ``count``,
    stopped at the first square), or None if there is none.  ``value_order``
    [n*n, n]: per cell, the order in which values are tried (random numbers
    drawn by the caller).  Raises if the search enters more than
    ``node_limit`` cells."""
    c = _square(n, cells)
    vo = None
    if value_order is not None:
        vo = np.ascontiguousarray(np.asarray(value_order, dtype=np.uint8).reshape(n * n, n))
    out = np.full(n * n, EMPTY, dtype=np.uint8)
    r = _load().oracle_first(n, int(bool(vs)), _u8(c), None if vo is None else _u8(vo), node_limit, _u8(out))
    if r < 0:
        raise ValueError("invalid oracle input or node limit reached")
    return out if r == 1 else None


def assignments(n: int, base, cells: Sequence[int], vs: bool = False) -> np.ndarray:
    """All consistent assignments of ``cells`` (flat indices i*n+j) extending
    ``base``, as full squares [K, n*n] (the workunits of Sec. 5.2)."""
    b = _square(n, base)
    c = (ctypes.c_int * max(1, len(cells)))(*cells)
    lib = _load()
    k = lib.oracle_assignments(n, int(bool(vs)), _u8(b), c, len(cells), None, 0)
    if k < 0:
        raise ValueError("invalid oracle input")
    out = np.zeros((k, n * n), dtype=np.uint8)
    if k:
        lib.oracle_assignments(n, int(bool(vs)), _u8(b), c, len(cells), _u8(out), k)
    return out


def total_from_fixed(n: int, fixed_count: int, vs: bool = False) -> int:
    """Undo the first-row normalisation.  Any relabelling of the values maps
    DLS to DLS bijectively (Sec. 2.2), so every first row occurs equally often
    and the total is N! times the fixed-first-row count.  For VS squares only
    relabellings that commute with v -> N-1-v keep the property; their number
    is 2^(N/2) (N/2)! for even N (a derived reading; the paper is silent)."""
    if vs:
        if n % 2 == 1:
            return fixed_count if n == 1 else 0
        m = n // 2
        return fixed_count * (2 ** m) * math.factorial(m)
    return fixed_count * math.factorial(n)


# --------------------------------------------------------------------------
# brute force over rows-as-permutations (a different construction)
# --------------------------------------------------------------------------

def brute_force_count(n: int, normalized: bool = True, vs: bool = False) -> int:
    """Count DLS of order n by stacking whole rows taken from the list of all
    permutations of 0..n-1 (the approach Sec. 2.1 describes and rejects as
    slow), checking columns and both diagonals.  Independent of the cell-by-
    cell search; only for n <= 6."""
    if n > 6:
        raise ValueError("brute force is for tiny orders only")
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.int64).reshape(-1, n)
    if vs:
        keep = np.all(perms + perms[:, ::-1] == n - 1, axis=1)
        perms = perms[keep]
    if perms.shape[0] == 0:
        return 0
    cols = np.arange(n)

    def rec(row: int, col_used: np.ndarray, md_used: np.ndarray, ad_used: np.ndarray) -> int:
        if row == n:
            return 1
        ok = ~np.any(col_used[cols[None, :], perms], axis=1)
        ok &= ~md_used[perms[:, row]]
        ok &= ~ad_used[perms[:, n - 1 - row]]
        total = 0
        for p in perms[ok]:
            cu = col_used.copy()
            cu[cols, p] = True
            mu = md_used.copy()
            mu[p[row]] = True
            au = ad_used.copy()
            au[p[n - 1 - row]] = True
            total += rec(row + 1, cu, mu, au)
        return total

    col_used = np.zeros((n, n), dtype=bool)
    md_used = np.zeros(n, dtype=bool)
    ad_used = np.zeros(n, dtype=bool)
    if normalized:
        first = np.arange(n)
        if vs and not np.all(first + first[::-1] == n - 1):
            return 0
        col_used[cols, first] = True
        md_used[first[0]] = True
        ad_used[first[n - 1]] = True
        return rec(1, col_used, md_used, ad_used)
    return rec(0, col_used, md_used, ad_used)


def is_dls(n: int, sq, vs: bool = False) -> bool:
    """Direct check of the definition of Sec. 1 on a full square."""
    a = np.asarray(sq, dtype=np.int64).reshape(n, n)
    full = set(range(n))
    if any(set(a[i, :]) != full for i in range(n)):
        return False
    if any(set(a[:, j]) != full for j in range(n)):
        return False
    if set(a[i, i] for i in range(n)) != full:
        return False
    if set(a[i, n - 1 - i] for i in range(n)) != full:
        return False
    if vs and not np.all(a + a[:, ::-1] == n - 1):
        return False
    return True


# --------------------------------------------------------------------------
# symmetry breaking (Sec. 4)
# --------------------------------------------------------------------------

def hourglass_group(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """All (p, q) of the hourglass-preserving M-transformations, built by
    closing generators under composition; T[i][j] = H[p[i]][q[j]]."""
    cap = 4096
    p = np.zeros(cap * n, dtype=np.int8)
    q = np.zeros(cap * n, dtype=np.int8)
    k = _load().oracle_hourglass_group(n, p.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                       q.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), cap)
    if k <= 0:
        raise ValueError("bad order")
    return p[:k * n].reshape(k, n).copy(), q[:k * n].reshape(k, n).copy()


def canon(n: int, design) -> int:
    """Algorithm 5: 0 if the design is not its class's lexicographically least
    member (row-major over known cells), else the class power."""
    r = _load().oracle_canon(n, _u8(_square(n, design)))
    if r < 0:
        raise ValueError("invalid design")
    return int(r)


def apply(n: int, g: int, design) -> np.ndarray:
    """Image of a design under group element g, renormalised by row 0."""
    out = np.zeros(n * n, dtype=np.uint8)
    if _load().oracle_apply(n, g, _u8(_square(n, design)), _u8(out)) != 0:
        raise ValueError("invalid design or element")
    return out


def hourglass_classes(n: int, vs: bool = False, threads: Optional[int] = None,
                      want_reps: bool = True):
    """Corollary 1, steps 1-2: every hourglass design of order n, split into
    classes.  Returns (n_hourglass, reps [C, n*n] sorted, mult [C])."""
    lib = _load()
    nh = ctypes.c_uint64(0)
    th = threads or default_threads()
    if not want_reps:
        c = lib.oracle_hourglass_classes(n, int(bool(vs)), None, None, 0, ctypes.byref(nh), th)
        if c < 0:
            raise ValueError("oracle failure")
        return int(nh.value), None, None
    cap = 1 << 16
    while True:
        reps = np.zeros((cap, n * n), dtype=np.uint8)
        mult = np.zeros(cap, dtype=np.uint32)
        c = lib.oracle_hourglass_classes(n, int(bool(vs)), _u8(reps),
                                         mult.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                         cap, ctypes.byref(nh), th)
        if c >= 0:
            break
        cap *= 4
        if cap > (1 << 26):
            raise ValueError("oracle failure")
    reps, mult = reps[:c], mult[:c]
    order = np.lexsort(reps.T[::-1])
    return int(nh.value), reps[order], mult[order]


def hourglass_cells(n: int) -> List[int]:
    """Cells of an hourglass design beyond row 0: rows 0 and n-1, the main
    diagonal and the antidiagonal (Sec. 4.2), as flat indices, row-major."""
    cells = set()
    for i in range(1, n):
        cells.add(i * n + i)
        cells.add(i * n + (n - 1 - i))
    for j in range(n):
        cells.add((n - 1) * n + j)
    return sorted(cells)


# --------------------------------------------------------------------------
# the cell order of Sec. 2.3
# --------------------------------------------------------------------------

def fill_order(n: int, assigned: Optional[Iterable[int]] = None, vs: bool = False,
               first: Optional[Iterable[int]] = None) -> List[int]:
    """Order in which the empty cells are filled (Sec. 2.3).

    At each step: if some row, column, main diagonal or antidiagonal has
    exactly n-1 assigned cells, its remaining cell comes next (the forced
    rule; the row-major-first such cell if there are several).  Otherwise the
    next cell is the one maximising V = r_i + c_j + md + ad (assigned cells in
    its row, its column, and on each diagonal it lies on), ties broken by
    row-major position.  Only the assigned/unassigned status of cells is used.

    ``vs``: only the left half (j < n/2) is filled; each pick also assigns its
    mirror (i, n-1-j), and a forced cell in the right half stands for its
    mirror.  ``first``: cells that must all come before any other cell (used
    to fill hourglass designs first, Sec. 4.3)."""
    assigned_set = set(range(n)) if assigned is None else set(assigned)
    a = np.zeros((n, n), dtype=bool)
    for c in assigned_set:
        a[c // n, c % n] = True
    pending_first = set(first) if first is not None else set()

    def lines(i, j):
        ls = [("r", i), ("c", j)]
        if i == j:
            ls.append(("md", 0))
        if i + j == n - 1:
            ls.append(("ad", 0))
        return ls

    def line_cells(kind, k):
        if kind == "r":
            return [(k, j) for j in range(n)]
        if kind == "c":
            return [(i, k) for i in range(n)]
        if kind == "md":
            return [(i, i) for i in range(n)]
        return [(i, n - 1 - i) for i in range(n)]

    def left(i, j):
        return (i, j) if not vs or 2 * j < n else (i, n - 1 - j)

    order: List[int] = []
    while True:
        empties = [(i, j) for i in range(n) for j in range(n) if not a[i, j]]
        if vs:
            empties = [(i, j) for (i, j) in empties if 2 * j <= n - 1]
        if not empties:
            break
        allowed = empties
        if pending_first:
            allowed = [(i, j) for (i, j) in empties if i * n + j in pending_first]
            if not allowed:
                pending_first = set()
                allowed = empties
        allowed_set = set(allowed)
        forced = []
        for kind in ("r", "c", "md", "ad"):
            for k in (range(n) if kind in ("r", "c") else [0]):
                cs = line_cells(kind, k)
                missing = [(i, j) for (i, j) in cs if not a[i, j]]
                if len(missing) == 1:
                    cell = left(*missing[0])
                    if cell in allowed_set:
                        forced.append(cell)
        if forced:
            pick = min(forced, key=lambda c: c[0] * n + c[1])
        else:
            best = None
            for (i, j) in allowed:
                v = a[i, :].sum() + a[:, j].sum()
                if i == j:
                    v += sum(a[t, t] for t in range(n))
                if i + j == n - 1:
                    v += sum(a[t, n - 1 - t] for t in range(n))
                if best is None or v > best[0]:
                    best = (v, (i, j))
            pick = best[1]
        i, j = pick
        a[i, j] = True
        if vs:
            a[i, n - 1 - j] = True
        order.append(i * n + j)
        pending_first.discard(i * n + j)
    return order


def count_assignments(n: int, base, cells: Sequence[int], vs: bool = False) -> int:
    """Number of consistent assignments of ``cells`` extending ``base``."""
    b = _square(n, base)
    c = (ctypes.c_int * max(1, len(cells)))(*cells)
    k = _load().oracle_assignments(n, int(bool(vs)), _u8(b), c, len(cells), None, 0)
    if k < 0:
        raise ValueError("invalid oracle input")
    return int(k)


def assignments_at(n: int, base, cells: Sequence[int], positions, vs: bool = False) -> np.ndarray:
    """The assignments ``assignments(n, base, cells, vs)`` would list at the
    given increasing positions, without storing the others."""
    b = _square(n, base)
    c = (ctypes.c_int * max(1, len(cells)))(*cells)
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int64))
    out = np.zeros((len(pos), n * n), dtype=np.uint8)
    r = _load().oracle_assignments_at(n, int(bool(vs)), _u8(b), c, len(cells),
                                      pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      len(pos), _u8(out))
    if r < 0:
        raise ValueError("invalid oracle input")
    return out
