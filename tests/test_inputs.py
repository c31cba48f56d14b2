"""The seeded graph generators: simple digraphs, exact sizes, reproducible,
and randomisation that keeps every in- and out-degree."""

import numpy as np
import pytest

from paper_1804_09741_amd import inputs as I


def _degrees(g):
    rp, cl = g
    n = len(rp) - 1
    return np.diff(rp), np.bincount(cl, minlength=n)


def test_workload_shapes():
    (g,) = I.workload_k3_er().graphs
    I.check_simple(*g)
    assert len(g[0]) == 201 and len(g[1]) == 800
    (g,) = I.workload_k4_chunglu().graphs
    I.check_simple(*g)
    assert len(g[0]) == 2001 and len(g[1]) == 10000
    out, inn = _degrees(g)
    assert out.max() <= 200 and inn.max() <= 200
    g = I.k5_batch_graph(0)
    assert len(g[0]) == 1001 and len(g[1]) == 3000
    g = I.k6_batch_graph(0)
    assert len(g[0]) == 701 and len(g[1]) == 1500
    assert np.diff(g[0]).max() <= 60


def test_reciprocity_fraction():
    (g,) = I.workload_k4_chunglu().graphs
    rp, cl = g
    s, d = I.arcs_from_csr(rp, cl)
    keys = set((s * 2000 + d).tolist())
    recip = sum(1 for a, b in zip(s.tolist(), d.tolist()) if b * 2000 + a in keys)
    # 10000 = 8333 base arcs + 1667 added reverses -> at least 3334 arcs in
    # pairs, plus the few pairs the base draw makes by chance
    assert 2 * (10000 - 8333) <= recip <= 2 * (10000 - 8333) + 100


@pytest.mark.parametrize("idx", [1, 2])
def test_randomisation_preserves_degrees(idx):
    for base, rnd in ((I.k5_batch_graph(0), I.k5_batch_graph(idx)),
                      (I.k6_batch_graph(0), I.k6_batch_graph(idx))):
        I.check_simple(*rnd)
        o0, i0 = _degrees(base)
        o1, i1 = _degrees(rnd)
        assert (o0 == o1).all() and (i0 == i1).all()
        assert not np.array_equal(base[1], rnd[1])


def test_seeded_reproducible():
    a = I.chung_lu_digraph(300, 900, 2.1, 50, 0.1, np.random.default_rng(3))
    b = I.chung_lu_digraph(300, 900, 2.1, 50, 0.1, np.random.default_rng(3))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_serving_stream_small():
    reqs = I.serving_requests(count=12, n_max=600)
    assert all(3 <= r.k <= 6 for r in reqs)
    assert all(b.arrival_s >= a.arrival_s for a, b in zip(reqs, reqs[1:]))
    for r in reqs:
        I.check_simple(*r.graph)
        n = len(r.graph[0]) - 1
        assert 100 <= n <= 600


def test_sparse_powerlaw_large_graph():
    """The vectorised recipe of the large graphs: simple, out-degrees in
    [0, 60] (repeated targets dropped), m about n times the mean out-degree
    of P(d) ~ d^-2.5 on [1, 60], reproducible."""
    n = 1 << 16
    g = I.sparse_powerlaw_digraph(n, 2.5, 60, np.random.default_rng(5))
    I.check_simple(*g)
    out = np.diff(g[0])
    assert out.max() <= 60 and out.min() >= 0
    d = np.arange(1, 61, dtype=np.float64)
    mean = float((d * d ** -2.5).sum() / (d ** -2.5).sum())
    assert abs(len(g[1]) / n - mean) < 0.05 * mean
    g2 = I.sparse_powerlaw_digraph(n, 2.5, 60, np.random.default_rng(5))
    assert np.array_equal(g[0], g2[0]) and np.array_equal(g[1], g2[1])
    w = I.workload_k6_large(1 << 14)
    assert w.k == 6 and len(w.graphs) == 1 and len(w.graphs[0][0]) == (1 << 14) + 1
