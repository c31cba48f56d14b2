"""The ensemble of random graphs and the per-class significance on the GPU,
against the oracle's switch chain (bit for bit) and z-scores (float64)."""

import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

pytestmark = pytest.mark.gpu


def _attempt_cap(target):
    return 8 * target + 1024


def _check_against_oracle(ctx, rp, col, count, seed, spa):
    g = ctx.load_graph(rp, col)
    made, acc = ctx.randomise(g, count, seed, spa)
    try:
        target = spa * len(col)
        for r, h in enumerate(made):
            exp_col, exp_acc = O.switch_chain(rp, col, seed, r, target, _attempt_cap(target))
            got_rp, got_col = h.read()
            assert np.array_equal(got_rp, np.asarray(rp, dtype=np.int32)), r
            assert np.array_equal(got_col, exp_col), (r, np.flatnonzero(got_col != exp_col)[:5])
            assert int(acc[r]) == exp_acc
            # the undirected degree the library recorded
            u = {(a, int(b)) for a in range(len(rp) - 1) for b in got_col[rp[a]:rp[a + 1]]}
            deg = np.zeros(len(rp) - 1, dtype=np.int64)
            for a, b in {tuple(sorted(x)) for x in u}:
                deg[a] += 1
                deg[b] += 1
            assert h.max_degree == int(deg.max(initial=0))
    finally:
        for h in made:
            h.free()
        g.free()


@pytest.mark.parametrize("seed", [1, 99])
def test_randomise_matches_oracle_small(ctx, seed):
    rng = np.random.default_rng([80, seed])
    rp, col = I.chung_lu_digraph(120, 480, 2.2, 30, 0.2, rng)
    _check_against_oracle(ctx, rp, col, count=4, seed=seed, spa=10)


def test_randomise_matches_oracle_tiny_graphs(ctx):
    """Few arcs: most rounds of 64 attempts hit arc slots already switched
    in the round, so the re-test path runs all the time."""
    rng = np.random.default_rng(84)
    for n, m in ((4, 3), (6, 8), (8, 16), (12, 30)):
        rp, col = I.er_digraph(n, m, rng)
        _check_against_oracle(ctx, rp, col, count=3, seed=n * 31 + m, spa=50)


def test_randomise_matches_oracle_k5_original(ctx):
    rp, col = I.k5_batch_graph(0)
    _check_against_oracle(ctx, rp, col, count=3, seed=2024, spa=10)


def test_randomise_edge_cases(ctx):
    rng = np.random.default_rng(81)
    rp, col = I.er_digraph(30, 90, rng)
    g = ctx.load_graph(rp, col)
    try:
        made, acc = ctx.randomise(g, 0, 1, 10)
        assert made == [] and len(acc) == 0
        made, acc = ctx.randomise(g, 2, 1, 0)      # no switches: the graph itself
        for h in made:
            assert np.array_equal(h.read()[1], col)
            h.free()
        assert not acc.any()
    finally:
        g.free()
    rp, col = I.complete_digraph(7)                # no valid switch
    g = ctx.load_graph(rp, col)
    try:
        made, acc = ctx.randomise(g, 2, 3, 5)
        for h in made:
            assert np.array_equal(h.read()[1], col)
            h.free()
        assert not acc.any()
    finally:
        g.free()


@pytest.mark.parametrize("k", [4, 5])
def test_random_graphs_count_like_host_loaded_copies(ctx, k):
    """The device-made graphs (their recorded |delta| sums size the batch
    workspace) count exactly like the same arcs loaded from the host."""
    rng = np.random.default_rng([82, k])
    rp, col = I.chung_lu_digraph(200, 800, 2.1, 40, 0.15, rng)
    g = ctx.load_graph(rp, col)
    made, _ = ctx.randomise(g, 3, 7, 10)
    t = ctx.table(k)
    copies = [ctx.load_graph(*h.read()) for h in made]
    try:
        h1, _ = ctx.count_batch(made, t)
        h2, _ = ctx.count_batch(copies, t)
        assert np.array_equal(h1, h2)
    finally:
        for h in made + copies + [g]:
            h.free()


def _gpu_significance(ctx, hist, nc):
    d_hist = torch.from_numpy(hist.astype(np.int64)).to("cuda:0")
    d_out = torch.zeros((3, nc), dtype=torch.float64, device="cuda:0")
    ctx.significance(d_hist, nc, d_out, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


def _assert_significance_equal(got, exp):
    fin = np.isfinite(exp)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.array_equal(got[~fin], exp[~fin])
    np.testing.assert_allclose(got[fin], exp[fin], rtol=1e-12, atol=1e-12)


def test_significance_closed_forms(ctx):
    R = 9
    h = np.zeros((R + 1, 4), dtype=np.uint64)
    h[1:, 0] = np.arange(1, R + 1)
    h[0, 0] = 20
    h[:, 1] = 7
    h[1:, 2] = 3
    h[0, 2] = 4
    h[1:, 3] = 3
    h[0, 3] = 1
    got = _gpu_significance(ctx, h, 4)
    assert got[0, 0] == (R + 1) / 2
    assert math.isclose(got[1, 0], math.sqrt(R * (R + 1) / 12), rel_tol=1e-14)
    assert (got[0, 1], got[1, 1], got[2, 1]) == (7, 0, 0)
    assert got[2, 2] == np.inf and got[2, 3] == -np.inf
    _assert_significance_equal(got, O.significance(h))
    with pytest.raises(M.MotifsError):
        _gpu_significance(ctx, h[:2], 4)


def test_pipeline_significance_matches_oracle(ctx):
    """Original + 20 random graphs, made on the device, counted in one batch,
    z-scores on the device; against the oracle's z-scores of the same
    histograms and the oracle's counts of the same random graphs."""
    k = 4
    rng = np.random.default_rng(83)
    rp, col = I.chung_lu_digraph(150, 600, 2.2, 30, 0.2, rng)
    g = ctx.load_graph(rp, col)
    made, _ = ctx.randomise(g, 20, 11, 10)
    t = ctx.table(k)
    try:
        b = ctx.batch([g] + made, t)
        try:
            d_hist = torch.zeros((21, t.num_classes), dtype=torch.int64, device="cuda:0")
            b.run(d_hist, torch.cuda.current_stream())
            d_out = torch.zeros((3, t.num_classes), dtype=torch.float64, device="cuda:0")
            ctx.significance(d_hist, t.num_classes, d_out, torch.cuda.current_stream())
            torch.cuda.synchronize()
            hist, _ = b.read()
        finally:
            b.free()
        _assert_significance_equal(d_out.cpu().numpy(), O.significance(hist))
        cc = t.class_codes()
        for r in (1, 20):
            exp_col, _ = O.switch_chain(rp, col, 11, r - 1, 10 * len(col), _attempt_cap(10 * len(col)))
            exp = O.count(rp, exp_col, k)
            got = {int(cc[i]): int(hist[r][i]) for i in np.flatnonzero(hist[r])}
            assert got == exp
    finally:
        for h in made + [g]:
            h.free()
