"""Both counting methods at the limits of LDS marks: MK_LDS_MARKS_MAX_VERTICES
vertices and a hub of degree up to MK_MAX_DEGREE, against the oracle where
it finishes in seconds and against closed forms where it would not.  (Larger
graphs, up to MK_MAX_VERTICES, are covered with the variants that keep the
marks in device memory.)"""

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

from gpu_helpers import as_code_dict

pytestmark = pytest.mark.gpu

METHODS = [M.METHOD_ESU, M.METHOD_CORES]
_EXPECTED = {}


def _oracle(key, g, k):
    """The oracle's histogram of a case, computed once for both methods."""
    if key not in _EXPECTED:
        _EXPECTED[key] = O.count(*g, k)
    return _EXPECTED[key]


def _count(ctx, g, k, method):
    gr = ctx.load_graph(*g)
    b = None
    try:
        b = ctx.batch([gr], ctx.table(k), method=method)
        b.run()
        hist, totals = b.read()
        return hist[0], int(totals[0])
    finally:
        if b is not None:
            b.free()
        gr.free()


def _max_n_with_hub(seed, hub_degree, extra_arcs):
    """MK_LDS_MARKS_MAX_VERTICES vertices: vertex 0 points at hub_degree
    others, plus random arcs among the rest."""
    n = M.MK_LDS_MARKS_MAX_VERTICES
    rng = np.random.default_rng(seed)
    src = [0] * hub_degree
    dst = list(range(1, hub_degree + 1))
    a = rng.integers(1, n, size=extra_arcs)
    b = rng.integers(1, n, size=extra_arcs)
    src += a.tolist()
    dst += b.tolist()
    keep = [(u, v) for u, v in dict.fromkeys(zip(src, dst)) if u != v]
    return I.csr_from_arcs(n, [u for u, _ in keep], [v for _, v in keep])


@pytest.mark.parametrize("method", METHODS)
def test_k3_max_vertices_and_hub(ctx, method):
    g = _max_n_with_hub(90, M.MK_MAX_DEGREE - 1, 12000)
    hist, total = _count(ctx, g, 3, method)
    assert total >= math.comb(M.MK_MAX_DEGREE - 1, 2)
    assert as_code_dict(hist, ctx.table(3).class_codes()) == _oracle("hub3", g, 3)


@pytest.mark.parametrize("k", [4, 5, 6])
@pytest.mark.parametrize("method", METHODS)
def test_max_vertices_sparse(ctx, k, method):
    rng = np.random.default_rng([91, k])
    g = I.er_digraph(M.MK_LDS_MARKS_MAX_VERTICES, 12000, rng)
    hist, _ = _count(ctx, g, k, method)
    assert as_code_dict(hist, ctx.table(k).class_codes()) == _oracle(("er", k), g, k)


@pytest.mark.parametrize("method", METHODS)
def test_k4_star_of_max_degree(ctx, method):
    """Out-star with MK_MAX_DEGREE leaves: C(4096, 3) = 11,444,858,880 4-sets,
    all in class 0 (beyond the oracle's reach; the closed form pins it)."""
    leaves = M.MK_MAX_DEGREE
    hist, total = _count(ctx, I.out_star(leaves), 4, method)
    assert total == math.comb(leaves, 3) and hist[0] == total


def test_degree_above_limit_rejected(ctx):
    with pytest.raises(M.MotifsError) as e:
        ctx.load_graph(*I.out_star(M.MK_MAX_DEGREE + 1))
    assert e.value.status == M.MK_ERANGE
