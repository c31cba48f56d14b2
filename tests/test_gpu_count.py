"""GPU enumeration (ESU) + lookup + histogram against the CPU oracle.

Small cases compare every class bit-exactly; closed-form graphs check the
known counts; batched, split and replayed runs must equal the plain run.
"""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

from gpu_helpers import as_code_dict, assert_hist_equals_oracle

pytestmark = pytest.mark.gpu


def _count(ctx, g, k, **opts):
    """H_k of one graph by the enumeration method (ESU)."""
    opts.setdefault("method", M.METHOD_ESU)
    gr = ctx.load_graph(*g)
    t = ctx.table(k)
    try:
        b = ctx.batch([gr], t, **opts)
        try:
            b.run()
            hist, totals = b.read()
            assert b.stats()["method"] == opts["method"]
            return hist[0], int(totals[0])
        finally:
            b.free()
    finally:
        gr.free()


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_count_entry_point(ctx, k):
    """mk_count (the library's method choice) equals the enumeration."""
    rng = np.random.default_rng([900, k])
    g = I.chung_lu_digraph(60, 200, 2.2, 20, 0.2, rng)
    gr = ctx.load_graph(*g)
    try:
        hist, total = ctx.count(gr, ctx.table(k))
    finally:
        gr.free()
    ref, ref_total = _count(ctx, g, k)
    assert np.array_equal(hist, ref) and total == ref_total


@pytest.mark.parametrize("k", [3, 4, 5, 6])
@pytest.mark.parametrize("seed", range(3))
def test_random_small_graphs(ctx, k, seed):
    rng = np.random.default_rng([1000, k, seed])
    n = int(rng.integers(20, 80))
    m = int(rng.integers(n, 4 * n))
    g = I.chung_lu_digraph(n, m, float(rng.uniform(2.0, 2.6)), 25, 0.2, rng)
    hist, total = _count(ctx, g, k)
    cc = ctx.table(k).class_codes()
    assert total == int(hist.sum())
    assert_hist_equals_oracle(hist, cc, *g, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_brute_force_tiny(ctx, k):
    rng = np.random.default_rng([2000, k])
    cc = ctx.table(k).class_codes()
    for _ in range(4):
        g = I.er_digraph(9, int(rng.integers(9, 30)), rng)
        hist, _ = _count(ctx, g, k)
        assert as_code_dict(hist, cc) == O.brute_force_count(*g, k)


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_closed_forms(ctx, k):
    t = ctx.table(k)
    full = (1 << (k * (k - 1))) - 1
    star = (1 << (k - 1)) - 1
    hist, total = _count(ctx, I.complete_digraph(9), k)
    assert total == math.comb(9, k) and hist[t.lookup(full)] == total
    hist, total = _count(ctx, I.out_star(40), k)
    assert total == math.comb(40, k - 1) and hist[0] == total and t.class_code(0) == star
    hist, total = _count(ctx, I.in_star(40), k)
    assert total == math.comb(40, k - 1) and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.directed_cycle(30), k)
    assert total == 30 and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.directed_path(30), k)
    assert total == 30 - k + 1 and np.count_nonzero(hist) == 1
    hist, total = _count(ctx, I.bidirected_cycle(30), k)
    assert total == 30 and np.count_nonzero(hist) == 1


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_hub_star_splits(ctx, k):
    """A hub of degree 300 (k=6: 60) forces second-level work splitting."""
    leaves = 300 if k < 6 else 60
    rng = np.random.default_rng([3000, k])
    s = [0] * leaves + rng.integers(1, leaves + 1, size=leaves // 3).tolist()
    d = list(range(1, leaves + 1)) + rng.integers(1, leaves + 1, size=leaves // 3).tolist()
    keep = [(a, b) for a, b in dict.fromkeys(zip(s, d)) if a != b]
    g = I.csr_from_arcs(leaves + 1, [a for a, _ in keep], [b for _, b in keep])
    cc = ctx.table(k).class_codes()
    h1, t1 = _count(ctx, g, k)
    h2, t2 = _count(ctx, g, k, split_threshold=1)
    h3, t3 = _count(ctx, g, k, split_threshold=1 << 40, waves_per_cu=1)
    assert np.array_equal(h1, h2) and np.array_equal(h1, h3)
    if k <= 5 or leaves <= 60:
        assert_hist_equals_oracle(h1, cc, *g, k)


def test_edge_cases(ctx):
    for k in (3, 4, 5, 6):
        t = ctx.table(k)
        for g in (I.empty_graph(0), I.empty_graph(5), I.complete_digraph(k - 1),
                  I.directed_path(k - 1), I.empty_graph(1)):
            hist, total = _count(ctx, g, k)
            assert total == 0 and hist.shape == (t.num_classes,) and not hist.any()
        hist, total = _count(ctx, I.complete_digraph(k), k)
        assert total == 1


def test_bad_graphs_rejected(ctx):
    cases = [
        ([0, 1, 1], [0], M.MK_EGRAPH),            # loop
        ([0, 2, 2], [1, 1], M.MK_EGRAPH),         # repeated arc
        ([0, 1, 1], [5], M.MK_EGRAPH),            # head out of range
        ([0, 2, 1], [1, 0], M.MK_EGRAPH),         # row_ptr decreases
        ([1, 1, 1], [], M.MK_EGRAPH),             # row_ptr[0] != 0
    ]
    for rp, cl, status in cases:
        with pytest.raises(M.MotifsError) as e:
            ctx.load_graph(np.array(rp, np.int32), np.array(cl + [0], np.int32))
        assert e.value.status == status
    n = M.MK_MAX_VERTICES + 1
    with pytest.raises(M.MotifsError) as e:
        ctx.load_graph(np.zeros(n + 1, np.int32), np.zeros(1, np.int32))
    assert e.value.status == M.MK_ERANGE


def test_batch_equals_plain_and_replays(ctx):
    k = 4
    rng = np.random.default_rng(77)
    graphs = [I.chung_lu_digraph(int(rng.integers(30, 300)), int(rng.integers(100, 900)), 2.2,
                                 40, 0.2, rng) for _ in range(9)]
    graphs.append(I.empty_graph(3))
    t = ctx.table(k)
    loaded = [ctx.load_graph(*g) for g in graphs]
    try:
        plain = [ctx.count(g, t)[0] for g in loaded]
        hb, tb = ctx.count_batch(loaded, t)
        for i in range(len(graphs)):
            assert np.array_equal(hb[i], plain[i])
            assert int(tb[i]) == int(plain[i].sum())
        b = ctx.batch(loaded, t)
        try:
            for rep in range(3):
                b.run()
                h, _ = b.read()
                assert np.array_equal(h, hb), rep
                _ = ctx.count(loaded[0], t)   # eager work between replays
        finally:
            b.free()
    finally:
        for g in loaded:
            g.free()


def test_torch_buffer_and_stream(ctx):
    torch = pytest.importorskip("torch")
    k = 3
    g = I.er_digraph(100, 400, np.random.default_rng(5))
    gr = ctx.load_graph(*g)
    t = ctx.table(k)
    try:
        b = ctx.batch([gr], t)
        out = torch.zeros((1, t.num_classes), dtype=torch.int64, device="cuda:0")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())  # the zeros land first
        b.run(out, stream=s)
        s.synchronize()
        h = out.cpu().numpy().astype(np.uint64)
        ref, _ = ctx.count(gr, t)
        assert np.array_equal(h[0], ref)
        b.free()
    finally:
        gr.free()


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_counting_paths_agree(ctx, k):
    """The per-wave hash, its constant-flush and bypass paths, and different
    queue grab sizes all give the same histogram (and the oracle's)."""
    rng = np.random.default_rng([4000, k])
    g = I.chung_lu_digraph(300, 1000, 2.1, 60 if k < 6 else 20, 0.15, rng)
    ref, _ = _count(ctx, g, k)
    for opts in ({"debug_flags": 1}, {"debug_flags": 2}, {"units_per_grab": 1},
                 {"units_per_grab": 64}, {"split_threshold": 1, "units_per_grab": 3},
                 {"units_per_wave": 4}, {"units_per_wave": 128, "split_threshold": 128}):
        h, _ = _count(ctx, g, k, **opts)
        assert np.array_equal(h, ref), opts
    if k <= 5:
        assert_hist_equals_oracle(ref, ctx.table(k).class_codes(), *g, k)


def test_autotune_keeps_results(ctx):
    k = 5
    rng = np.random.default_rng(4100)
    graphs = [I.chung_lu_digraph(200, 700, 2.2, 50, 0.1, rng) for _ in range(4)]
    t = ctx.table(k)
    loaded = [ctx.load_graph(*g) for g in graphs]
    try:
        opts, ms, dms = ctx.autotune(loaded, t, trials=1)
        assert ms > 0
        ref, _ = ctx.count_batch(loaded, t)
        b = ctx.batch(loaded, t, **opts)
        try:
            b.run()
            h, _ = b.read()
        finally:
            b.free()
        assert np.array_equal(h, ref)
    finally:
        for g in loaded:
            g.free()


@pytest.mark.parametrize("method", [M.METHOD_ESU, M.METHOD_CORES])
def test_graph_replays_equal_eager(ctx, method):
    """The captured pass -- the preparation (use_graph 1) or the whole pass,
    preparation, counting kernel and finish (use_graph 2): every replay,
    with eager work and host synchronisation between replays, equals the
    eager pass; the timing events give the pass (and, with 1, the kernel)
    durations; a new histogram buffer is captured anew."""
    rng = np.random.default_rng(4200)
    graphs = [I.chung_lu_digraph(int(rng.integers(100, 400)), int(rng.integers(300, 1200)),
                                 2.2, 40, 0.1, rng) for _ in range(4)]
    k = 5
    t = ctx.table(k)
    loaded = [ctx.load_graph(*g) for g in graphs]
    try:
        eager = ctx.batch(loaded, t, method=method, use_graph=-1)
        try:
            eager.run()
            ref, _ = eager.read()
        finally:
            eager.free()
        for use_graph in (1, 2):
            _replays(ctx, loaded, t, method, use_graph, ref)
    finally:
        for g in loaded:
            g.free()


def _replays(ctx, loaded, t, method, use_graph, ref):
    import torch
    b = ctx.batch(loaded, t, method=method, use_graph=use_graph)
    try:
        for buf in range(2):
            d = torch.full((len(loaded), t.num_classes), 3, dtype=torch.int64, device="cuda:0")
            for _ in range(3):
                b.run(d, torch.cuda.current_stream())
                pass_ms, kern_ms = b.timing()
                assert pass_ms > 0
                assert (0 < kern_ms <= pass_ms) if use_graph == 1 else kern_ms == -1
                assert np.array_equal(d.cpu().numpy().astype(np.uint64), ref)
                h, _ = ctx.count(loaded[buf], t)  # eager work between replays
                assert np.array_equal(h, ref[buf])
                d.fill_(5)
    finally:
        b.free()
