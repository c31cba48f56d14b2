"""Pins of the oracle's pieces for counting from connected (k-2)-sets
(Section 3, the counting loop over L_{k-2}): the core multiplicity of a
class, the raw pair sums, and the step-by-step reference of the loop."""

import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I


def code_of(k, arcs):
    c = 0
    for i, j in arcs:
        c |= 1 << O.bit_of(k, i, j)
    return c


def complete(k):
    return code_of(k, [(i, j) for i in range(k) for j in range(k) if i != j])


def out_star(k):
    return code_of(k, [(0, j) for j in range(1, k)])


def in_star(k):
    return code_of(k, [(j, 0) for j in range(1, k)])


def dpath(k):
    return code_of(k, [(i, i + 1) for i in range(k - 1)])


def dcycle(k):
    return code_of(k, [(i, (i + 1) % k) for i in range(k)])


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_core_mult_closed_forms(k):
    # every (k-2)-subset of a complete digraph is a core
    assert O.core_mult(k, complete(k)) == math.comb(k, 2)
    # a path has one core: its inner k-2 vertices
    assert O.core_mult(k, dpath(k)) == 1
    # a star's cores hold the centre and k-3 of the k-1 leaves
    assert O.core_mult(k, out_star(k)) == math.comb(k - 1, 2)
    assert O.core_mult(k, in_star(k)) == math.comb(k - 1, 2)
    # a cycle's cores are its k runs of k-2 consecutive vertices
    # (k = 3: the triangle, every vertex touches both others)
    assert O.core_mult(k, dcycle(k)) == k


def test_core_mult_hand_example():
    # k = 4: triangle 0,1,2 with vertex 3 hanging off 0.  Cores (connected
    # pairs whose complement both touch them): {0,1}, {0,2}, {0,3}; not
    # {1,2}, which vertex 3 does not touch
    g = code_of(4, [(0, 1), (1, 2), (2, 0), (0, 3)])
    assert O.core_mult(4, g) == 3


@pytest.mark.parametrize("k", [3, 4])
def test_core_mult_zero_exactly_when_disconnected(k):
    for code in range(1 << (k * (k - 1))):
        m = O.core_mult(k, code)
        assert (m > 0) == O.connected(k, code), code
        assert m <= math.comb(k, 2)


@pytest.mark.parametrize("k", [4, 5, 6])
def test_core_mult_is_a_class_invariant(k):
    rng = np.random.default_rng([61, k])
    for _ in range(40):
        code = int(rng.integers(0, 1 << (k * (k - 1))))
        perm = rng.permutation(k)
        moved = 0
        for i in range(k):
            for j in range(k):
                if i != j and (code >> O.bit_of(k, i, j)) & 1:
                    moved |= 1 << O.bit_of(k, int(perm[i]), int(perm[j]))
        assert O.core_mult(k, code) == O.core_mult(k, moved)


def _tiny_graphs(k, count=4, n=7):
    rng = np.random.default_rng([62, k])
    out = [I.out_star(5), I.directed_cycle(6), I.bidirected_cycle(5)]
    for _ in range(count):
        out.append(I.er_digraph(n, int(rng.integers(n, 3 * n)), rng))
    return out


@pytest.mark.parametrize("k", [3, 4, 5])
def test_raw_pair_sums_are_core_mult_times_counts(k):
    # the raw sums over (X, {y, z}) are a different computation from both
    # the class counts (all k-subsets) and the per-class multiplicity
    for g in _tiny_graphs(k):
        raw = O.core_pairs_count(*g, k)
        hist = O.brute_force_count(*g, k)
        assert raw == {c: O.core_mult(k, c) * v for c, v in hist.items()}


@pytest.mark.parametrize("k", [3, 4, 5])
def test_raw_pair_sums_complete_digraph(k):
    # K_n: C(n, k-2) cores, each with C(n-k+2, 2) pairs, all of one class;
    # and C(n, k-2) C(n-k+2, 2) = C(n, k) C(k, 2)
    n = 7
    raw = O.core_pairs_count(*I.complete_digraph(n), k)
    total = math.comb(n, k - 2) * math.comb(n - k + 2, 2)
    assert raw == {complete(k): total}
    assert total == math.comb(n, k) * math.comb(k, 2)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_algorithm1_equals_brute_force(k):
    for g in _tiny_graphs(k):
        assert O.algorithm1_count(*g, k) == O.brute_force_count(*g, k)


def test_algorithm1_k6_small():
    rng = np.random.default_rng(63)
    for g in (I.er_digraph(8, 14, rng), I.out_star(6), I.directed_cycle(7)):
        assert O.algorithm1_count(*g, 6) == O.brute_force_count(*g, 6)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_algorithm1_equals_esu_oracle(k):
    rng = np.random.default_rng([64, k])
    g = I.chung_lu_digraph(12, 30, 2.2, 6, 0.2, rng)
    assert O.algorithm1_count(*g, k) == O.count(*g, k)


def test_paper_motif_figure():
    """Section 2's figure of motif(v, A(v), B(v)): the cells are read off the
    A/B/C definitions, and the loop over L_1 = {v, a, b} counts the one
    3-set in the class of that figure."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "paper_fig_motif_example.json")) as f:
        fig = json.load(f)
    idx = {name: i for i, name in enumerate(fig["vertices"])}
    arcs = {(idx[u], idx[v]) for u, v in fig["arcs"]}
    v = idx["v"]
    # A(v): arcs both ways; B(v): v -> u only; C(v): u -> v only
    for name, cell in fig["cells"].items():
        u = idx[name]
        got = {(True, True): "A", (True, False): "B", (False, True): "C"}[((v, u) in arcs,
                                                                          (u, v) in arcs)]
        assert got == cell
    rp, col = I.csr_from_arcs(3, [a for a, _ in sorted(arcs)], [b for _, b in sorted(arcs)])
    code = code_of(3, sorted(arcs))
    expected = {O.canon(3, code): 1}
    assert O.algorithm1_count(rp, col, 3) == expected == O.brute_force_count(rp, col, 3)
    # one cell pair (A, B) with weight 1 * 1 and no arc between a and b;
    # the class has one core: {v} touches both a and b, {a} and {b} do not
    assert O.core_pairs_count(rp, col, 3) == expected
    assert O.core_mult(3, code) == 1
