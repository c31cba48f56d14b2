"""The single-graph workloads past the LDS limit at their full size, in the
launch configuration the benchmark times: k = 6 on the power-law digraph of
2^20 vertices (1.6e10 connected 6-sets) and k = 7 on the one of 2^17
vertices (3.0e10 connected 7-sets).  The oracle does not finish on them, so
the results are checked through properties that hold at any size: a
relabelled copy has the same histogram (roots, extension lists, hub splits
and the order of the work all change), a different split threshold cuts the
hubs into different work units with the same result, and every k = 7 class
is reported under its canonical code (the oracle's canon7)."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

pytestmark = pytest.mark.gpu


def _count6(ctx, t, g, **opts):
    loaded = ctx.load_graph(*g)
    b = None
    try:
        b = ctx.batch([loaded], t, **opts)
        b.run()
        hist, totals = b.read()
        return hist[0], int(totals[0]), b.stats()
    finally:
        if b is not None:
            b.free()
        loaded.free()


def test_k6_large_relabel_and_split(ctx):
    w = I.workload_k6_large()
    g = w.graphs[0]
    n = len(g[0]) - 1
    assert n == M.MK_MAX_VERTICES
    t = ctx.table(6)
    hist, total, st = _count6(ctx, t, g)
    assert st["adjacency"] == M.ADJ_LISTS and st["marks"] == M.MARKS_GLOBAL
    assert total == int(hist.sum()) > 10 ** 10
    print("k6 large: %d subgraphs, %d classes, %d units" % (
        total, int(np.count_nonzero(hist)), st["units"]), flush=True)
    rg = I.relabel(*g, np.random.default_rng(9500).permutation(n))
    hist_r, total_r, _ = _count6(ctx, t, rg)
    assert total_r == total
    assert np.array_equal(hist_r, hist)
    # a split floor far above the adaptive threshold: fewer, larger units
    # over the hubs
    hist_s, _, st_s = _count6(ctx, t, g, split_threshold=1 << 24)
    assert st_s["units"] < st["units"]
    assert np.array_equal(hist_s, hist)


def test_k7_large_relabel_and_canonical(ctx):
    w = I.workload_k6_large(1 << 17)
    g = w.graphs[0]
    n = len(g[0]) - 1
    rg = I.relabel(*g, np.random.default_rng(9501).permutation(n))
    loaded = [ctx.load_graph(*x) for x in (g, rg)]
    try:
        out, totals, _ = ctx.count7(loaded)
    finally:
        for x in loaded:
            x.free()
    (codes, counts), (codes_r, counts_r) = out
    assert int(totals[0]) == int(totals[1]) == int(counts.sum()) > 10 ** 10
    assert np.array_equal(codes, codes_r) and np.array_equal(counts, counts_r)
    assert np.all(counts > 0) and np.all(np.diff(codes.astype(np.int64)) > 0)
    print("k7 large: %d subgraphs, %d classes" % (int(totals[0]), len(codes)), flush=True)
    for c in codes.tolist():
        assert O.canon7(c) == c
