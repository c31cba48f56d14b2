"""mk_count_static (no allocation: the library's static device scratch)
gives mk_count's histogram, on two calls in a row with the second graph
smaller than the first (the scratch keeps the first call's contents), for
k = 3..6; graphs past its limits are refused before any launch."""

import numpy as np
import pytest

from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

pytestmark = pytest.mark.gpu


def _static(ctx, g, t):
    import torch
    d = torch.full((t.num_classes,), 7, dtype=torch.int64, device="cuda:0")
    # on the stream that wrote the 7s: the library's clear and counts follow
    # them (on another stream the fill could land after the counts)
    ctx.count_static(g, t, d, torch.cuda.current_stream())
    return d.cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_static_equals_count_twice(ctx, k):
    rng = np.random.default_rng([9900, k])
    big = I.chung_lu_digraph(900, 3200, 2.2, 60, 0.2, rng)
    small = I.chung_lu_digraph(120, 300, 2.4, 20, 0.1, rng)
    t = ctx.table(k)
    for spec in (big, small):
        g = ctx.load_graph(*spec)
        try:
            ref, total = ctx.count(g, t)
            got = _static(ctx, g, t)
            assert np.array_equal(got, ref)
            assert int(got.sum()) == total > 0
        finally:
            g.free()


def test_static_k6_batch_graphs(ctx):
    """Graphs of the k = 6 batch one after another (larger, then smaller)."""
    w = I.workload_k6_batch()
    t = ctx.table(6)
    order = sorted(range(4), key=lambda i: -len(w.graphs[i][1]))
    for i in order:
        g = ctx.load_graph(*w.graphs[i])
        try:
            ref, _ = ctx.count(g, t)
            assert np.array_equal(_static(ctx, g, t), ref)
        finally:
            g.free()


def test_static_degenerate_and_limits(ctx):
    t = ctx.table(4)
    g = ctx.load_graph(*I.empty_graph(3))
    try:
        assert not _static(ctx, g, t).any()
    finally:
        g.free()
    # too many vertices for LDS marks: refused on the host
    big = I.er_digraph(M.MK_LDS_MARKS_MAX_VERTICES + 1, 20000, np.random.default_rng(3))
    g = ctx.load_graph(*big)
    try:
        with pytest.raises(M.MotifsError) as e:
            _static(ctx, g, t)
        assert e.value.status == M.MK_ERANGE
    finally:
        g.free()
    # workspace beyond the static array: refused on the host
    n = M.MK_LDS_MARKS_MAX_VERTICES
    rng = np.random.default_rng(4)
    src = np.repeat(np.arange(n), 400)
    dst = (src + 1 + rng.integers(0, n - 1, size=len(src))) % n
    key = np.unique(src.astype(np.int64) * n + dst)
    dense = I.csr_from_arcs(n, key // n, key % n)
    assert len(dense[1]) * 40 > M.mk_static_scratch_bytes()
    g = ctx.load_graph(*dense)
    try:
        with pytest.raises(M.MotifsError) as e:
            _static(ctx, g, t)
        assert e.value.status == M.MK_ERANGE
    finally:
        g.free()
