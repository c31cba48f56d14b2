"""Pins of the oracle's k = 7 histograms (keyed by canonical code): the
pure-Python brute force over all 7-subsets, closed forms, and invariants.
None of them re-uses the oracle's C code."""

import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I

K = 7


def _code_of_arcs(arcs):
    """Code of a 7-vertex digraph given by its arcs (i, j)."""
    return sum(1 << O.bit_of(K, i, j) for i, j in arcs)


def _py_canon7(code):
    a = [[i != j and bool((code >> O.bit_of(K, i, j)) & 1) for j in range(K)] for i in range(K)]
    return O._py_canon(K, a)


def _random_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    pairs = set()
    while len(pairs) < m:
        u, v = (int(x) for x in rng.integers(0, n, size=2))
        if u != v:
            pairs.add((u, v))
    pairs = sorted(pairs)
    return I.csr_from_arcs(n, [u for u, _ in pairs], [v for _, v in pairs])


@pytest.mark.parametrize("seed,n,m", [(1, 9, 18), (2, 9, 26), (3, 10, 16)])
def test_brute_force_tiny(seed, n, m):
    g = _random_graph(n, m, [7000, seed])
    assert O.count(*g, K) == O.brute_force_count(*g, K)


def test_canon7_against_python_and_invariants():
    rng = np.random.default_rng(7001)
    for _ in range(4):
        code = int(rng.integers(0, 1 << 42))
        c = O.canon7(code)
        assert c == _py_canon7(code)
    for _ in range(40):
        code = int(rng.integers(0, 1 << 42)) & int(rng.integers(0, 1 << 42))
        c = O.canon7(code)
        assert c <= code and O.canon7(c) == c
        p = rng.permutation(K)
        relabeled = sum(1 << O.bit_of(K, int(p[i]), int(p[j]))
                        for i in range(K) for j in range(K)
                        if i != j and (code >> O.bit_of(K, i, j)) & 1)
        assert O.canon7(relabeled) == c


def test_closed_forms():
    full = (1 << 42) - 1
    assert O.count(*I.complete_digraph(9), K) == {full: math.comb(9, 7)}
    # out-star: the centre first, its arcs at bits 0..5 -- the smallest
    # connected code
    assert O.count(*I.out_star(8), K) == {63: math.comb(8, 6)}
    # in-star: the centre last, arcs i -> 6 at bits 6i + 5
    in_star = sum(1 << (6 * i + 5) for i in range(6))
    assert O.count(*I.in_star(8), K) == {in_star: math.comb(8, 6)}
    path7 = _py_canon7(_code_of_arcs([(i, i + 1) for i in range(6)]))
    cycle7 = _py_canon7(_code_of_arcs([(i, (i + 1) % 7) for i in range(7)]))
    bipath7 = _py_canon7(_code_of_arcs([(i, i + 1) for i in range(6)] +
                                       [(i + 1, i) for i in range(6)]))
    assert O.count(*I.directed_cycle(10), K) == {path7: 10}
    assert O.count(*I.directed_cycle(7), K) == {cycle7: 1}
    assert O.count(*I.directed_path(12), K) == {path7: 6}
    assert O.count(*I.bidirected_cycle(9), K) == {bipath7: 9}
    assert O.count(*I.empty_graph(20), K) == {}
    assert O.count(*I.directed_path(6), K) == {}


def test_relabel_union_and_reverse():
    rng = np.random.default_rng(7002)
    g = I.chung_lu_digraph(30, 55, 2.2, 8, 0.2, rng)
    h = O.count(*g, K)
    assert sum(h.values()) > 0 and len(h) > 5
    assert O.count(*I.relabel(*g, rng.permutation(30)), K) == h
    h2 = O.count(*I.disjoint_union([g, g]), K)
    assert h2 == {c: 2 * v for c, v in h.items()}
    # reversing every arc maps each class to the class of its transpose
    rev = {}
    for c, v in h.items():
        t = sum(1 << O.bit_of(K, j, i) for i in range(K) for j in range(K)
                if i != j and (c >> O.bit_of(K, i, j)) & 1)
        t = O.canon7(t)
        rev[t] = rev.get(t, 0) + v
    assert O.count(*I.reverse(*g), K) == rev


def test_total_is_connected_7_sets():
    g = _random_graph(12, 22, 7003)
    n, arcs, delta = O._arcs_and_delta(*g)
    expected = sum(1 for sub in itertools.combinations(range(n), K)
                   if O._weakly_connected(sub, delta))
    assert sum(O.count(*g, K).values()) == expected
