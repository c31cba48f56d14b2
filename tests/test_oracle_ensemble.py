"""Pins of the oracle's ensemble of random graphs (degree-preserving directed
switches drawing from SplitMix64) and of its per-class significance."""

import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_values():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.json")) as f:
        g = json.load(f)
    got = [O.splitmix64(g["seed"], i) for i in range(len(g["outputs_hex"]))]
    assert got == [int(x, 16) for x in g["outputs_hex"]]


def _in_degrees(n, col):
    return np.bincount(np.asarray(col, dtype=np.int64), minlength=n)


def _arcs(row_ptr, col):
    rp = np.asarray(row_ptr)
    return {(u, int(col[t])) for u in range(len(rp) - 1) for t in range(rp[u], rp[u + 1])}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_switches_keep_degrees_and_simplicity(seed):
    rng = np.random.default_rng([70, seed])
    rp, col = I.chung_lu_digraph(60, 240, 2.2, 20, 0.2, rng)
    m = len(col)
    new, acc = O.switch_chain(rp, col, seed, 0, 10 * m, 100 * m)
    assert acc == 10 * m
    assert np.array_equal(_in_degrees(60, new), _in_degrees(60, col))
    arcs = _arcs(rp, new)
    assert len(arcs) == m                                # no duplicate
    assert all(u != v for u, v in arcs)                  # no loop
    # out-degrees: every arc keeps its row; most heads have moved
    assert np.mean(new != col) > 0.5


def test_one_switch_is_a_swap_of_heads():
    rng = np.random.default_rng(71)
    rp, col = I.er_digraph(12, 30, rng)
    new, acc = O.switch_chain(rp, col, 5, 3, 1, 1000)
    assert acc == 1
    diff = np.flatnonzero(new != col)
    assert len(diff) == 2
    i, j = diff
    assert new[i] == col[j] and new[j] == col[i]


def test_zero_target_and_no_valid_switch():
    rng = np.random.default_rng(72)
    rp, col = I.er_digraph(20, 50, rng)
    new, acc = O.switch_chain(rp, col, 9, 0, 0, 1000)
    assert acc == 0 and np.array_equal(new, col)
    # complete digraph: every switch would duplicate an arc
    rp, col = I.complete_digraph(6)
    new, acc = O.switch_chain(rp, col, 9, 0, 50, 5000)
    assert acc == 0 and np.array_equal(new, col)
    # out-star: every pair of arcs shares its tail
    rp, col = I.out_star(10)
    new, acc = O.switch_chain(rp, col, 9, 0, 50, 5000)
    assert acc == 0 and np.array_equal(new, col)


def test_streams_differ_by_graph_and_seed():
    rng = np.random.default_rng(73)
    rp, col = I.er_digraph(40, 120, rng)
    a, _ = O.switch_chain(rp, col, 11, 0, 200, 10000)
    b, _ = O.switch_chain(rp, col, 11, 1, 200, 10000)
    c, _ = O.switch_chain(rp, col, 12, 0, 200, 10000)
    a2, _ = O.switch_chain(rp, col, 11, 0, 200, 10000)
    assert np.array_equal(a, a2)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_significance_closed_forms():
    R = 9
    h = np.zeros((R + 1, 4), dtype=np.uint64)
    h[1:, 0] = np.arange(1, R + 1)       # 1..R: mean (R+1)/2, var R(R+1)/12
    h[0, 0] = 20
    h[:, 1] = 7                          # constant: std 0, H_0 = mean -> z 0
    h[1:, 2] = 3                         # std 0, H_0 > mean -> +inf
    h[0, 2] = 4
    h[1:, 3] = 3                         # std 0, H_0 < mean -> -inf
    h[0, 3] = 1
    mean, std, z = O.significance(h)
    assert mean[0] == (R + 1) / 2
    assert math.isclose(std[0], math.sqrt(R * (R + 1) / 12), rel_tol=1e-15)
    assert math.isclose(z[0], (20 - (R + 1) / 2) / math.sqrt(R * (R + 1) / 12), rel_tol=1e-15)
    assert (mean[1], std[1], z[1]) == (7, 0, 0)
    assert z[2] == np.inf and z[3] == -np.inf
    with pytest.raises(ValueError):
        O.significance(h[:2])
