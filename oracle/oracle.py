"""Python front end of the CPU oracle for Motifs-k.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liboracle.so`` (plain C,
built from ``oracle.c`` with gcc) and adds a second, pure-Python brute-force
checker for tiny graphs.  Nothing here is shared with the HIP library.

Conventions (Section 3.2 of the paper: the isomorphism key is the adjacency
matrix of the k-vertex subgraph):

* code of an ordered vertex tuple (s_0..s_{k-1}): bit i(k-1) + j - [j > i]
  is set iff the arc s_i -> s_j exists;
* canonical code of a class: the minimum code over all k! relabelings;
* class id (k <= 5 here): rank of the canonical code among the canonical
  codes of weakly connected k-vertex digraphs.  The paper numbers classes
  1..|P_k| without fixing an order; ranking by canonical code is our choice.
"""

from __future__ import annotations

import ctypes
import functools
import itertools
import os
import subprocess
from typing import Dict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               _SRC, "-o", _LIB])
    return _LIB


def load_library(path: str):
    """A ctypes handle on an oracle library built from oracle.c (or from a
    deliberately broken copy of it, for the mutation tests)."""
    lib = ctypes.CDLL(path)
    lib.oracle_connected.restype = ctypes.c_int
    lib.oracle_connected.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_canon.restype = ctypes.c_uint32
    lib.oracle_canon.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_canon_table.restype = ctypes.c_int
    lib.oracle_canon_table.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_core_mult.restype = ctypes.c_int
    lib.oracle_core_mult.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_splitmix64.restype = ctypes.c_uint64
    lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_switch_chain.restype = ctypes.c_int64
    lib.oracle_switch_chain.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_void_p]
    lib.oracle_count.restype = ctypes.c_int64
    lib.oracle_count.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.oracle_canon7.restype = ctypes.c_uint64
    lib.oracle_canon7.argtypes = [ctypes.c_uint64]
    lib.oracle_count7.restype = ctypes.c_int64
    lib.oracle_count7.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p]
    return lib


@functools.lru_cache(maxsize=None)
def _lib():
    if not os.path.exists(_LIB):
        build()
    return load_library(_LIB)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error %d" % code)
        self.code = code


def bit_of(k: int, i: int, j: int) -> int:
    return i * (k - 1) + j - (1 if j > i else 0)


def connected(k: int, code: int) -> bool:
    return bool(_lib().oracle_connected(k, code))


def canon(k: int, code: int) -> int:
    return int(_lib().oracle_canon(k, code))


def canon_table_with(lib, k: int):
    """(canon, conn) from a given oracle library."""
    n = 1 << (k * (k - 1))
    c = np.empty(n, dtype=np.uint32)
    ok = np.empty(n, dtype=np.uint8)
    rc = lib.oracle_canon_table(k, c.ctypes.data, ok.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    c.setflags(write=False)
    ok.setflags(write=False)
    return c, ok


@functools.lru_cache(maxsize=None)
def canon_table(k: int):
    """(canon, conn): canonical code and connectivity of every code, k <= 5."""
    return canon_table_with(_lib(), k)


@functools.lru_cache(maxsize=None)
def class_codes(k: int) -> np.ndarray:
    """Canonical codes of the weakly connected classes, ascending (k <= 5)."""
    c, ok = canon_table(k)
    out = np.unique(c[ok.astype(bool)])
    out.setflags(write=False)
    return out


def count(row_ptr, col, k: int) -> Dict[int, int]:
    """H_k as {canonical code: count} (zero classes omitted); k = 3..7."""
    if k == 7:
        return count7_with(_lib(), row_ptr, col)
    return count_with(_lib(), row_ptr, col, k, canon_table(k)[0] if 3 <= k <= 5 else None)


def canon7(code: int) -> int:
    """Canonical form of a 7-vertex code (minimum over the 5040 relabelings)."""
    return int(_lib().oracle_canon7(code))


def count7_with(lib, row_ptr, col) -> Dict[int, int]:
    """H_7 as {canonical code: count} from a given oracle library."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = len(row_ptr) - 1
    cap = 1 << 14
    while True:
        codes = np.zeros(cap, dtype=np.uint64)
        counts = np.zeros(cap, dtype=np.uint64)
        total = ctypes.c_uint64(0)
        rc = lib.oracle_count7(n, row_ptr.ctypes.data, col.ctypes.data if len(col) else None,
                               codes.ctypes.data, counts.ctypes.data, cap, ctypes.byref(total))
        if rc == -5:
            cap *= 4
            continue
        if rc < 0:
            raise OracleError(int(rc))
        return {int(c): int(v) for c, v in zip(codes[:rc], counts[:rc])}


def count_with(lib, row_ptr, col, k: int, table=None) -> Dict[int, int]:
    """H_k from a given oracle library (table: its canon table for k <= 5)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = len(row_ptr) - 1
    tptr = None
    if 3 <= k <= 5:
        tptr = table.ctypes.data
    cap = 1 << 16
    while True:
        codes = np.zeros(cap, dtype=np.uint32)
        counts = np.zeros(cap, dtype=np.uint64)
        total = ctypes.c_uint64(0)
        rc = lib.oracle_count(n, row_ptr.ctypes.data, col.ctypes.data if len(col) else None,
                                 k, tptr, codes.ctypes.data, counts.ctypes.data, cap,
                                 ctypes.byref(total))
        if rc == -5:
            cap *= 4
            continue
        if rc < 0:
            raise OracleError(int(rc))
        return {int(c): int(v) for c, v in zip(codes[:rc], counts[:rc])}


def dense_hist(row_ptr, col, k: int) -> np.ndarray:
    """H_k as a dense uint64 vector indexed by class id (k <= 5)."""
    cc = class_codes(k)
    h = np.zeros(len(cc), dtype=np.uint64)
    for code, v in count(row_ptr, col, k).items():
        i = int(np.searchsorted(cc, code))
        assert i < len(cc) and cc[i] == code
        h[i] = v
    return h


def core_mult(k: int, code: int) -> int:
    """Cores of the k-vertex digraph `code`: (k-2)-subsets X with G[X] weakly
    connected that both remaining vertices touch (see oracle.c)."""
    r = int(_lib().oracle_core_mult(k, code))
    if r < 0:
        raise OracleError(r)
    return r


@functools.lru_cache(maxsize=None)
def core_mult_table(k: int) -> np.ndarray:
    """core_mult of every class, in class-id order (k <= 5)."""
    out = np.array([core_mult(k, int(c)) for c in class_codes(k)], dtype=np.uint8)
    out.setflags(write=False)
    return out


# --------------------------------------------------------------------------
# ensemble of random graphs and significance (Section 1, steps (a) and (c))
# --------------------------------------------------------------------------

def splitmix64(seed: int, i: int) -> int:
    """Output i of SplitMix64 seeded with `seed` (see oracle.c)."""
    return int(_lib().oracle_splitmix64(seed & (2**64 - 1), i))


def switch_chain(row_ptr, col, seed: int, r: int, target: int, max_attempts: int):
    """(new col, accepted): graph r of the ensemble with this seed (oracle.c
    states the switch rule).  row_ptr is unchanged."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    out = np.empty(max(len(col), 1), dtype=np.int32)
    acc = _lib().oracle_switch_chain(len(row_ptr) - 1, row_ptr.ctypes.data,
                                     col.ctypes.data if len(col) else None, seed, r, target,
                                     max_attempts, out.ctypes.data)
    if acc < 0:
        raise OracleError(int(acc))
    return out[:len(col)], int(acc)


def significance(hist) -> np.ndarray:
    """(mean, std, z) per class, float64, of an ensemble's histograms: row 0
    is the original graph, rows 1..R its random graphs (R >= 2).  mean and
    the sample standard deviation (divisor R - 1) are over the random graphs;
    z = (H_0 - mean) / std, with z = 0 where std = 0 and H_0 = mean and an
    infinity of H_0 - mean's sign where std = 0 otherwise (Section 1, step
    (c); the paper names no statistic, this is the usual z-score)."""
    h = np.asarray(hist, dtype=np.uint64)
    if h.ndim != 2 or h.shape[0] < 3:
        raise ValueError("need the original and at least two random graphs")
    rnd = h[1:].astype(np.float64)
    mean = rnd.sum(axis=0) / rnd.shape[0]
    var = ((rnd - mean) ** 2).sum(axis=0) / (rnd.shape[0] - 1)
    std = np.sqrt(var)
    diff = h[0].astype(np.float64) - mean
    z = np.zeros_like(mean)
    pos = std > 0
    z[pos] = diff[pos] / std[pos]
    z[~pos & (diff > 0)] = np.inf
    z[~pos & (diff < 0)] = -np.inf
    return np.stack([mean, std, z])


# --------------------------------------------------------------------------
# second, independent brute force (tiny graphs only)
# --------------------------------------------------------------------------

def _py_canon(k: int, a) -> int:
    best = None
    for p in itertools.permutations(range(k)):
        c = 0
        for i in range(k):
            for j in range(k):
                if i != j and a[i][j]:
                    c |= 1 << bit_of(k, p[i], p[j])
        if best is None or c < best:
            best = c
    return best


def brute_force_count(row_ptr, col, k: int) -> Dict[int, int]:
    """H_k by the definition: every k-subset, kept if weakly connected."""
    row_ptr = np.asarray(row_ptr)
    n = len(row_ptr) - 1
    arcs = set()
    for u in range(n):
        for t in range(row_ptr[u], row_ptr[u + 1]):
            arcs.add((u, int(col[t])))
    out: Dict[int, int] = {}
    for sub in itertools.combinations(range(n), k):
        a = [[(sub[i], sub[j]) in arcs for j in range(k)] for i in range(k)]
        seen, stack = {0}, [0]
        while stack:
            u = stack.pop()
            for w in range(k):
                if w not in seen and (a[u][w] or a[w][u]):
                    seen.add(w)
                    stack.append(w)
        if len(seen) != k:
            continue
        c = _py_canon(k, a)
        out[c] = out.get(c, 0) + 1
    return out


def _arcs_and_delta(row_ptr, col):
    row_ptr = np.asarray(row_ptr)
    n = len(row_ptr) - 1
    arcs = set()
    for u in range(n):
        for t in range(row_ptr[u], row_ptr[u + 1]):
            arcs.add((u, int(col[t])))
    delta = [set() for _ in range(n)]
    for u, v in arcs:
        delta[u].add(v)
        delta[v].add(u)
    return n, arcs, delta


def _weakly_connected(vs, delta) -> bool:
    vs = list(vs)
    seen, stack = {vs[0]}, [vs[0]]
    while stack:
        u = stack.pop()
        for w in vs:
            if w not in seen and w in delta[u]:
                seen.add(w)
                stack.append(w)
    return len(seen) == len(vs)


def _canon_of(sub, arcs, k):
    return _py_canon(k, [[(sub[i], sub[j]) in arcs for j in range(k)] for i in range(k)])


def core_pairs_count(row_ptr, col, k: int) -> Dict[int, int]:
    """By definition, for tiny graphs: over every connected (k-2)-set X and
    every unordered pair {y, z} of vertices of adj(X), count the class of
    G[X + {y, z}] -- the raw sum that the (k-2)-set counting of Section 3
    forms before any division."""
    n, arcs, delta = _arcs_and_delta(row_ptr, col)
    out: Dict[int, int] = {}
    for X in itertools.combinations(range(n), k - 2):
        if not _weakly_connected(X, delta):
            continue
        adj = sorted(set().union(*(delta[x] for x in X)) - set(X))
        for y, z in itertools.combinations(adj, 2):
            c = _canon_of(list(X) + [y, z], arcs, k)
            out[c] = out.get(c, 0) + 1
    return out


def algorithm1_count(row_ptr, col, k: int) -> Dict[int, int]:
    """Section 3's counting from L_{k-2}, step by step, for tiny graphs.

    For each connected (k-2)-set X: partition adj(X) into cells by each
    vertex's A/B/C/N relation to every member of X (Section 2); for every
    unordered pair of cells {Y, Z} add C(|Y|, 2) (Y = Z) or |Y| |Z| to the
    class of motif(X, Y, Z) -- X plus one vertex of each cell, no arc between
    the two; then, for every pair u, v of adj(X) joined by an arc, add one to
    the class of G[X + {u, v}] and take one from motif(X, cell(u), cell(v)).
    Every connected k-set S is reached once per core of S, so the raw sums
    are divided by core_mult of the class at the end.
    """
    n, arcs, delta = _arcs_and_delta(row_ptr, col)
    raw: Dict[int, int] = {}

    def add(c, w):
        raw[c] = raw.get(c, 0) + w

    def motif_code(X, ty, tz):
        # vertices 0..k-3 = X, k-2 = a vertex of cell ty, k-1 = of cell tz;
        # a cell is a tuple of (arc member -> vertex, arc vertex -> member)
        a = [[False] * k for _ in range(k)]
        for i in range(k - 2):
            for j in range(k - 2):
                a[i][j] = i != j and (X[i], X[j]) in arcs
        for p, t in ((k - 2, ty), (k - 1, tz)):
            for i in range(k - 2):
                a[i][p], a[p][i] = t[i]
        return _py_canon(k, a)

    for X in itertools.combinations(range(n), k - 2):
        if not _weakly_connected(X, delta):
            continue
        adj = sorted(set().union(*(delta[x] for x in X)) - set(X))
        cell_of = {u: tuple(((x, u) in arcs, (u, x) in arcs) for x in X) for u in adj}
        cells: Dict[tuple, int] = {}
        for u in adj:
            cells[cell_of[u]] = cells.get(cell_of[u], 0) + 1
        keys = sorted(cells)
        for i, ty in enumerate(keys):
            for tz in keys[i:]:
                w = cells[ty] * (cells[ty] - 1) // 2 if ty == tz else cells[ty] * cells[tz]
                if w:
                    add(motif_code(X, ty, tz), w)
        for u, v in itertools.combinations(adj, 2):
            if (u, v) in arcs or (v, u) in arcs:
                add(_canon_of(list(X) + [u, v], arcs, k), 1)
                add(motif_code(X, cell_of[u], cell_of[v]), -1)
    out: Dict[int, int] = {}
    for c, r in raw.items():
        if r == 0:
            continue
        m = core_mult(k, c)
        if r < 0:
            raise ValueError("raw count of class %d is negative" % c)
        if m == 0 or r % m:
            raise ValueError("raw count %d of class %d is not a multiple of %d" % (r, c, m))
        out[c] = r // m
    return out
