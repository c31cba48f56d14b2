"""Code-formation variants of the enumeration and graphs past the LDS marks
limit: arc tests on the sorted typed lists (MK_ADJ_LISTS, no bit matrix;
Algorithms 2-5 of Section 3.1 test pairs, scan lists, or split by degree),
per-wave marks in device memory (MK_MARKS_GLOBAL), and graphs with up to
MK_MAX_VERTICES vertices.  Every variant is compared with the oracle bit
for bit; where the oracle would not finish, a disjoint union of copies of a
small graph (scattered over the whole id range) pins the result through the
oracle's count of one copy."""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

from gpu_helpers import as_code_dict, assert_hist_equals_oracle

pytestmark = pytest.mark.gpu

VARIANTS = [
    # (method, adjacency, marks)
    (M.METHOD_ESU, M.ADJ_BITS, M.MARKS_LDS),
    (M.METHOD_ESU, M.ADJ_LISTS, M.MARKS_LDS),
    (M.METHOD_ESU, M.ADJ_LISTS, M.MARKS_GLOBAL),
    (M.METHOD_CORES, M.ADJ_LISTS, M.MARKS_LDS),
]


def _run(ctx, graphs, k, **opts):
    loaded = [ctx.load_graph(*g) for g in graphs]
    b = None
    try:
        b = ctx.batch(loaded, ctx.table(k), **opts)
        b.run()
        hist, totals = b.read()
        st = b.stats()
        b.run()  # a replay of the captured preparation gives the same counts
        hist2, _ = b.read()
        assert np.array_equal(hist, hist2)
        return hist, totals, st
    finally:
        if b is not None:
            b.free()
        for g in loaded:
            g.free()


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("variant", VARIANTS, ids=["esu-bits-lds", "esu-lists-lds",
                                                   "esu-lists-global", "cores-lists-lds"])
def test_variants_random_batch(ctx, k, variant):
    method, adj, marks = variant
    rng = np.random.default_rng([7100, k])
    # k = 6 by the core method on sorted lists: smaller graphs, so that the
    # oracle's 6-sets stay few (the core method's per-core cells and arc
    # pairs are the same code path at any size)
    n_hi, m_hi = (80, 220) if (method == M.METHOD_CORES and k == 6) else (160, 500)
    graphs = [I.chung_lu_digraph(int(rng.integers(20, n_hi)), int(rng.integers(60, m_hi)),
                                 float(rng.uniform(2.0, 2.6)), 30, 0.2, rng) for _ in range(5)]
    graphs.append(I.empty_graph(4))
    graphs.append(I.complete_digraph(k + 2))
    hist, totals, st = _run(ctx, graphs, k, method=method, adjacency=adj, marks=marks)
    assert (st["method"], st["adjacency"], st["marks"]) == variant
    cc = ctx.table(k).class_codes()
    for i, g in enumerate(graphs):
        assert_hist_equals_oracle(hist[i], cc, *g, k)
        assert int(totals[i]) == int(hist[i].sum())


@pytest.mark.parametrize("k", [3, 4])
def test_lists_hub_of_max_degree(ctx, k):
    """A vertex with MK_MAX_DEGREE neighbours, half of them bidirected: its
    raw out + in list (6144 entries) is sorted in one workgroup."""
    d = M.MK_MAX_DEGREE
    n = d + 1
    src = [0] * d + list(range(1, d // 2 + 1))
    dst = list(range(1, d + 1)) + [0] * (d // 2)
    rng = np.random.default_rng(7200)
    a = rng.integers(1, n, size=1500)
    b = rng.integers(1, n, size=1500)
    arcs = [(u, v) for u, v in dict.fromkeys(zip(src + a.tolist(), dst + b.tolist())) if u != v]
    g = I.csr_from_arcs(n, [u for u, _ in arcs], [v for _, v in arcs])
    h_lists, t_lists, st = _run(ctx, [g], k, method=M.METHOD_ESU, adjacency=M.ADJ_LISTS,
                                marks=M.MARKS_GLOBAL)
    assert st["adjacency"] == M.ADJ_LISTS
    if k == 3:
        assert_hist_equals_oracle(h_lists[0], ctx.table(k).class_codes(), *g, k)
    else:
        # C(4096, 3) 4-sets around the hub alone: beyond the oracle; the
        # bit-matrix variant and the closed form of the star part pin it
        h_bits, _, _ = _run(ctx, [g], k, method=M.METHOD_ESU, adjacency=M.ADJ_BITS)
        assert np.array_equal(h_bits, h_lists)
        assert int(t_lists[0]) >= math.comb(d, 3)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_beyond_lds_marks_limit(ctx, k):
    """n = 3 x MK_LDS_MARKS_MAX_VERTICES: the library switches to list-built
    adjacency, global marks and enumeration by itself."""
    n = 3 * M.MK_LDS_MARKS_MAX_VERTICES
    rng = np.random.default_rng([7300, k])
    if k <= 4:
        g = I.chung_lu_digraph(n, 40000, 2.3, 40, 0.1, rng)
    else:  # sparser, so that the oracle finishes in seconds
        g = I.er_digraph(n, 30000 if k == 5 else 25000, rng)
    hist, _, st = _run(ctx, [g], k)
    assert (st["method"], st["adjacency"], st["marks"]) == (M.METHOD_ESU, M.ADJ_LISTS,
                                                            M.MARKS_GLOBAL)
    assert_hist_equals_oracle(hist[0], ctx.table(k).class_codes(), *g, k)


def _scattered_copies(small, copies, n, rng):
    """`copies` disjoint copies of `small` plus isolated vertices up to n,
    vertex ids shuffled over [0, n)."""
    u = I.disjoint_union([small] * copies)
    nu = len(u[0]) - 1
    g = I.disjoint_union([u, I.empty_graph(n - nu)])
    return I.relabel(*g, rng.permutation(n))


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_max_vertices_scattered_copies(ctx, k):
    """MK_MAX_VERTICES vertices: 3000 copies of a small random graph spread
    over the whole id range; each class counts 3000 x the oracle's count
    of one copy."""
    rng = np.random.default_rng([7400, k])
    small = I.chung_lu_digraph(60, 150, 2.2, 20, 0.2, rng)
    g = _scattered_copies(small, 3000, M.MK_MAX_VERTICES, rng)
    hist, totals, st = _run(ctx, [g], k)
    assert st["marks"] == M.MARKS_GLOBAL
    exp = {c: 3000 * v for c, v in O.count(*small, k).items()}
    assert as_code_dict(hist[0], ctx.table(k).class_codes()) == exp
    assert int(totals[0]) == sum(exp.values())


def test_mixed_batch_small_and_big(ctx):
    """One batch with a graph past the LDS limit: every graph of it runs the
    global-marks variant, each with its own histogram."""
    k = 4
    rng = np.random.default_rng(7500)
    graphs = [I.chung_lu_digraph(300, 900, 2.2, 30, 0.2, rng),
              I.er_digraph(M.MK_LDS_MARKS_MAX_VERTICES + 1000, 20000, rng),
              I.empty_graph(0),
              I.directed_cycle(9)]
    hist, totals, st = _run(ctx, graphs, k)
    assert st["marks"] == M.MARKS_GLOBAL and st["adjacency"] == M.ADJ_LISTS
    cc = ctx.table(k).class_codes()
    for i, g in enumerate(graphs):
        assert_hist_equals_oracle(hist[i], cc, *g, k)


def test_variant_option_errors(ctx):
    big = ctx.load_graph(*I.er_digraph(M.MK_LDS_MARKS_MAX_VERTICES + 1, 100,
                                       np.random.default_rng(7600)))
    small = ctx.load_graph(*I.directed_cycle(10))
    t = ctx.table(4)
    try:
        for gr, opts, status in [
            (big, dict(marks=M.MARKS_LDS), M.MK_ERANGE),
            (big, dict(method=M.METHOD_CORES), M.MK_ERANGE),
            (small, dict(marks=M.MARKS_GLOBAL, adjacency=M.ADJ_BITS), M.MK_EINVAL),
            (small, dict(adjacency=3), M.MK_EINVAL),
            (small, dict(marks=-1), M.MK_EINVAL),
            (small, dict(units_per_wave=-1), M.MK_EINVAL),
            (small, dict(units_per_wave=5000), M.MK_EINVAL),
        ]:
            with pytest.raises(M.MotifsError) as e:
                ctx.batch([gr], t, **opts)
            assert e.value.status == status, opts
        with pytest.raises(M.MotifsError) as e:
            ctx.randomise(big, 1, 1)
        assert e.value.status == M.MK_ERANGE
        with pytest.raises(M.MotifsError) as e:
            ctx.batch([small], t, debug_flags=8)
        assert e.value.status == M.MK_EINVAL
    finally:
        big.free()
        small.free()


def test_autotune_tries_adjacency(ctx):
    rng = np.random.default_rng(7700)
    graphs = [ctx.load_graph(*I.chung_lu_digraph(400, 1500, 2.2, 40, 0.2, rng))
              for _ in range(3)]
    try:
        best, ms, dms = ctx.autotune(graphs, ctx.table(5), trials=1)
        assert best["adjacency"] in (M.ADJ_AUTO, M.ADJ_BITS, M.ADJ_LISTS) and ms > 0
    finally:
        for g in graphs:
            g.free()
