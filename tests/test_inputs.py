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
