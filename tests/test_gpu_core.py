"""The (k-2)-set counting method (Section 3's loop over L_{k-2}) on the GPU:
its per-class divisors against the oracle's, and its histograms against the
oracle and against the enumeration method, bit for bit."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

from gpu_helpers import as_code_dict, assert_hist_equals_oracle

pytestmark = pytest.mark.gpu


def _count(ctx, g, k, **opts):
    opts.setdefault("method", M.METHOD_CORES)
    gr = ctx.load_graph(*g)
    b = ctx.batch([gr], ctx.table(k), **opts)
    try:
        b.run()
        hist, totals = b.read()
        assert b.stats()["method"] == opts["method"]
        return hist[0], int(totals[0])
    finally:
        b.free()
        gr.free()


@pytest.mark.parametrize("k", [3, 4, 5])
def test_core_mult_table_matches_oracle(ctx, k):
    assert np.array_equal(ctx.table(k).core_mult(), O.core_mult_table(k))


def test_core_mult_table_k6(ctx):
    t = ctx.table(6)
    m = t.core_mult()
    cc = t.class_codes()
    assert len(m) == t.num_classes == 1530843
    assert m.min() >= 1 and m.max() <= 15
    assert m[0] == math.comb(5, 2) and m[-1] == 15  # out-star, complete digraph
    rng = np.random.default_rng(5000)
    for i in rng.choice(len(cc), size=3000, replace=False):
        assert int(m[i]) == O.core_mult(6, int(cc[i])), i
    part = t.core_mult(1000, 24)
    assert np.array_equal(part, m[1000:1024])


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("seed", range(3))
def test_cores_random_small_graphs(ctx, k, seed):
    rng = np.random.default_rng([5100, k, seed])
    n = int(rng.integers(20, 80))
    m = int(rng.integers(n, 4 * n))
    g = I.chung_lu_digraph(n, m, float(rng.uniform(2.0, 2.6)), 25, 0.2, rng)
    hist, total = _count(ctx, g, k)
    assert total == int(hist.sum())
    assert_hist_equals_oracle(hist, ctx.table(k).class_codes(), *g, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_cores_brute_force_tiny(ctx, k):
    rng = np.random.default_rng([5200, k])
    cc = ctx.table(k).class_codes()
    for _ in range(4):
        g = I.er_digraph(9, int(rng.integers(9, 30)), rng)
        hist, _ = _count(ctx, g, k)
        assert as_code_dict(hist, cc) == O.brute_force_count(*g, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_cores_closed_forms(ctx, k):
    t = ctx.table(k)
    full = (1 << (k * (k - 1))) - 1
    hist, total = _count(ctx, I.complete_digraph(9), k)
    assert total == math.comb(9, k) and hist[t.lookup(full)] == total
    hist, total = _count(ctx, I.out_star(40), k)
    assert total == math.comb(40, k - 1) and hist[0] == total
    hist, total = _count(ctx, I.in_star(40), k)
    assert total == math.comb(40, k - 1) and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.directed_cycle(30), k)
    assert total == 30 and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.directed_path(30), k)
    assert total == 30 - k + 1 and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.bidirected_cycle(30), k)
    assert total == 30 and np.count_nonzero(hist) == 1


def test_cores_edge_cases(ctx):
    for k in (3, 4, 5, 6):
        t = ctx.table(k)
        for g in (I.empty_graph(0), I.empty_graph(5), I.complete_digraph(k - 1),
                  I.directed_path(k - 1), I.empty_graph(1)):
            hist, total = _count(ctx, g, k)
            assert total == 0 and hist.shape == (t.num_classes,) and not hist.any()
        hist, total = _count(ctx, I.complete_digraph(k), k)
        assert total == 1


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_cores_hub_and_counting_paths(ctx, k):
    """A hub graph, counted with splitting, hash bypass, flush-always and
    small grabs: every variant equals the enumeration method's result."""
    rng = np.random.default_rng([5300, k])
    g = I.chung_lu_digraph(300, 1000, 2.1, 60 if k < 6 else 20, 0.15, rng)
    ref, _ = _count(ctx, g, k, method=M.METHOD_ESU)
    for opts in ({}, {"debug_flags": 1}, {"debug_flags": 2}, {"debug_flags": 4},
                 {"units_per_grab": 1},
                 {"split_threshold": 1, "units_per_grab": 3},
                 {"split_threshold": 1 << 40, "waves_per_cu": 1}):
        h, _ = _count(ctx, g, k, **opts)
        assert np.array_equal(h, ref), opts
    if k <= 5:
        assert_hist_equals_oracle(ref, ctx.table(k).class_codes(), *g, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_cores_hub_star(ctx, k):
    """A star of degree 300 (k=6: 60) plus random arcs: one huge cell."""
    leaves = 300 if k < 6 else 60
    rng = np.random.default_rng([5400, k])
    s = [0] * leaves + rng.integers(1, leaves + 1, size=leaves // 3).tolist()
    d = list(range(1, leaves + 1)) + rng.integers(1, leaves + 1, size=leaves // 3).tolist()
    keep = [(a, b) for a, b in dict.fromkeys(zip(s, d)) if a != b]
    g = I.csr_from_arcs(leaves + 1, [a for a, _ in keep], [b for _, b in keep])
    h1, _ = _count(ctx, g, k)
    h2, _ = _count(ctx, g, k, method=M.METHOD_ESU)
    assert np.array_equal(h1, h2)


@pytest.mark.parametrize("k", [5, 6])
def test_cores_dense_parent_overflows_arc_list(ctx, k):
    """K_70: a parent's adj(P) holds over 2,048 arc pairs, so the cores fall
    back to scanning every vertex's list; the count is still C(70, k)."""
    t = ctx.table(k)
    hist, total = _count(ctx, I.complete_digraph(70), k)
    assert total == math.comb(70, k)
    assert hist[t.lookup((1 << (k * (k - 1))) - 1)] == total


def _batch(ctx, graphs, t, **opts):
    b = ctx.batch(graphs, t, **opts)
    try:
        b.run()
        b.run()  # a replay of the captured graph must give the same
        return b.read()
    finally:
        b.free()


@pytest.mark.parametrize("k", [5, 6])
def test_cores_equal_esu_on_workload_batches(ctx, k):
    w = I.workload_k5_batch(count=21) if k == 5 else I.workload_k6_batch()
    t = ctx.table(k)
    loaded = [ctx.load_graph(*g) for g in w.graphs]
    try:
        h_esu, tot_esu = _batch(ctx, loaded, t, method=M.METHOD_ESU)
        h_core, tot_core = _batch(ctx, loaded, t, method=M.METHOD_CORES)
        assert np.array_equal(h_core, h_esu)
        assert np.array_equal(tot_core, tot_esu)
        assert_hist_equals_oracle(h_core[0], t.class_codes(), *w.graphs[0], k)
    finally:
        for g in loaded:
            g.free()
