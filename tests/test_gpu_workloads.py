"""The five workloads at full size, in the launch configuration the
benchmark times, every graph compared with the oracle bit for bit.

The oracle's histograms of every graph (all 101 of the k = 5 batch, all 31
of the k = 6 batch, k = 7 on those 31, and every request of the serving
stream whose size estimate is at most 1e8 subgraphs) are stored as digests
in ``tests/golden/oracle_digests.json``, written by
``tests/golden/make_oracle_digests.py`` (oracle and seeded generators only:
about 6,000 CPU-seconds, too long for a test run).  Each GPU histogram is
serialised the same way and its digest compared; the graph's own digest is
checked first, so a drift of the generators is reported as such.  On a
mismatch the oracle recomputes that graph to show the classes that differ.
The small single-graph configs are also compared densely with the oracle
run live."""

import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I

from gpu_helpers import as_code_dict, assert_hist_equals_oracle
from oracle.digest import dense_digest, graph_digest, pairs_digest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_digests.json")


@pytest.fixture(scope="module")
def digests():
    with open(GOLDEN) as f:
        return json.load(f)


def _check_input(rec, g, what):
    assert rec["graph"] == graph_digest(*g), (
        "%s: the seeded generator no longer gives the graph the stored oracle "
        "result was computed from" % what)


def _explain(got, g, k, what):
    """Only on a mismatch: the oracle's own count, to name the classes."""
    exp = O.count(*g, k)
    keys = sorted(set(got) | set(exp))
    bad = [(c, got.get(c, 0), exp.get(c, 0)) for c in keys if got.get(c, 0) != exp.get(c, 0)]
    return "%s: %d classes differ from the oracle, first (code, gpu, oracle): %s" % (
        what, len(bad), bad[:5])


def _check_dense(rec, hist, cc, g, k, what):
    if dense_digest(hist, cc) != rec["hist"]:
        pytest.fail(_explain(as_code_dict(hist, cc), g, k, what))
    assert int(hist.sum()) == rec["total"]


def test_k3_er_full(ctx, digests):
    w = I.workload_k3_er()
    rec = digests[w.name][0]
    _check_input(rec, w.graphs[0], w.name)
    t = ctx.table(3)
    g = ctx.load_graph(*w.graphs[0])
    hist, total = ctx.count(g, t)
    g.free()
    assert total == int(hist.sum()) > 0
    assert np.array_equal(hist, O.dense_hist(*w.graphs[0], 3))
    _check_dense(rec, hist, t.class_codes(), w.graphs[0], 3, w.name)


def test_k4_chunglu_full(ctx, digests):
    w = I.workload_k4_chunglu()
    rec = digests[w.name][0]
    _check_input(rec, w.graphs[0], w.name)
    t = ctx.table(4)
    g = ctx.load_graph(*w.graphs[0])
    hist, total = ctx.count(g, t)
    g.free()
    assert np.array_equal(hist, O.dense_hist(*w.graphs[0], 4))
    _check_dense(rec, hist, t.class_codes(), w.graphs[0], 4, w.name)


def _batch_check(ctx, w, recs, plain_every, **opts):
    assert len(recs) == len(w.graphs)
    for i, g in enumerate(w.graphs):
        _check_input(recs[i], g, "%s graph %d" % (w.name, i))
    t = ctx.table(w.k)
    loaded = [ctx.load_graph(*g) for g in w.graphs]
    try:
        b = ctx.batch(loaded, t, **opts)
        try:
            b.run()
            hist, totals = b.read()
        finally:
            b.free()
        cc = t.class_codes()
        for i, g in enumerate(w.graphs):
            _check_dense(recs[i], hist[i], cc, g, w.k, "%s graph %d" % (w.name, i))
        assert np.all(totals == hist.sum(axis=1))
        # one graph per launch gives the same histograms
        for i in range(0, len(w.graphs), plain_every):
            h, tot = ctx.count(loaded[i], t)
            assert np.array_equal(h, hist[i]) and tot == int(totals[i])
    finally:
        for g in loaded:
            g.free()


def test_k5_batch_full(ctx, digests):
    """All 101 graphs, counted from the (k-2)-sets (the library's choice)."""
    w = I.workload_k5_batch()
    _batch_check(ctx, w, digests[w.name], plain_every=20)


def test_k5_batch_full_enumeration(ctx, digests):
    """All 101 graphs again, by enumeration of every 5-set."""
    from paper_1804_09741_amd import motifs as M
    w = I.workload_k5_batch()
    _batch_check(ctx, w, digests[w.name], plain_every=1000, method=M.METHOD_ESU)


def test_k6_batch_full(ctx, digests):
    """All 31 graphs, in the launch configuration the benchmark times."""
    w = I.workload_k6_batch()
    _batch_check(ctx, w, digests[w.name], plain_every=10)


def test_k7_batch_full(ctx, digests):
    """k = 7 on all 31 graphs of the k = 6 batch (classes by canonical
    code), twice: on a cold and then a warm canonical-code cache."""
    w = I.workload_k6_batch()
    recs = digests["k7_batch31_powerlaw_n700_m1500"]
    for i, g in enumerate(w.graphs):
        _check_input(recs[i], g, "k7 graph %d" % i)
    loaded = [ctx.load_graph(*g) for g in w.graphs]
    try:
        for _ in range(2):
            out, totals, _ = ctx.count7(loaded)
            for i, (codes, counts) in enumerate(out):
                if pairs_digest(codes, counts) != recs[i]["hist"]:
                    pytest.fail(_explain(dict(zip(codes.tolist(), counts.tolist())),
                                         w.graphs[i], 7, "k7 graph %d" % i))
                assert int(totals[i]) == recs[i]["total"]
    finally:
        for g in loaded:
            g.free()


def test_serving_stream_oracle(ctx, digests):
    """Every request of the serving stream (1,000 requests, k in 3..6, n up
    to 5,000) whose size estimate is at most 1e8 subgraphs, submitted to the
    server all at once so that they share the device, each compared with
    the oracle; the same requests counted alone give the same histograms."""
    chk = digests["serving"]["checked"]
    idx = sorted(int(i) for i in chk)
    assert len(idx) > 500
    reqs = [I.serving_request(i) for i in idx]
    for i, (k, g) in zip(idx, reqs):
        assert chk[str(i)]["k"] == k
        _check_input(chk[str(i)], g, "request %d" % i)
    tables = {k: ctx.table(k) for k in (3, 4, 5, 6)}
    ccs = {k: tables[k].class_codes() for k in tables}
    loaded = [ctx.load_graph(*g) for _, g in reqs]
    try:
        srv = ctx.server()
        try:
            tickets = [srv.submit(g, k) for g, (k, _) in zip(loaded, reqs)]
            served = [srv.wait(t, k)[0] for t, (k, _) in zip(tickets, reqs)]
        finally:
            srv.stop()
        for i, h, (k, g) in zip(idx, served, reqs):
            _check_dense(chk[str(i)], h, ccs[k], g, k, "request %d (k=%d)" % (i, k))
        for j in range(0, len(reqs), 8):
            h, _ = ctx.count(loaded[j], tables[reqs[j][0]])
            assert np.array_equal(h, served[j])
    finally:
        for g in loaded:
            g.free()
