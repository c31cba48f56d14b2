"""Continuous-batching server: every request's histogram equals the same
request solved alone (tolerance 0), including requests submitted while
others run; admission by footprint; timeouts and bad tickets."""

import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I
from paper_1804_09741_amd import motifs as M

from gpu_helpers import assert_hist_equals_oracle

pytestmark = pytest.mark.gpu


def _requests(seed, count, n_max=400):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(3, 7))
        n = int(rng.integers(30, n_max))
        m = int(round(n * rng.uniform(2.0, 4.0)))
        cap = 40 if k <= 5 else 15
        out.append((k, I.chung_lu_digraph(n, m, float(rng.uniform(2.0, 2.6)), cap, 0.1, rng)))
    return out


def test_served_equals_alone(ctx):
    reqs = _requests(1, 24)
    graphs = [ctx.load_graph(*g) for _, g in reqs]
    alone = [ctx.count(g, ctx.table(k))[0] for (k, _), g in zip(reqs, graphs)]
    srv = ctx.server(tick_units=64)
    try:
        # first half at once, second half while the first half runs
        tickets = [srv.submit(g, k) for (k, _), g in zip(reqs[:12], graphs[:12])]
        first = srv.wait(tickets[0], reqs[0][0])
        tickets += [srv.submit(g, k) for (k, _), g in zip(reqs[12:], graphs[12:])]
        results = [first] + [srv.wait(t, k) for t, (k, _) in zip(tickets[1:], reqs[1:])]
    finally:
        srv.stop()
    for (hist, times), ref, (k, g) in zip(results, alone, reqs):
        assert np.array_equal(hist, ref)
        assert times["submit_us"] <= times["admit_us"] <= times["done_us"]
    for (hist, _), (k, g) in list(zip(results, reqs))[:6]:
        assert_hist_equals_oracle(hist, ctx.table(k).class_codes(), *g, k)
    for g in graphs:
        g.free()


def test_groups_across_sizes_and_empty(ctx):
    """Requests admitted together are grouped by k and size class of n;
    every one equals its count alone, including graphs with no k-subgraph
    (a group with no work units) and one class per group."""
    rng = np.random.default_rng(9200)
    specs = [(4, I.chung_lu_digraph(n, 3 * n, 2.3, 40, 0.1, rng)) for n in (90, 700, 1500, 3000)]
    specs += [(4, I.empty_graph(2)), (4, I.empty_graph(50)), (5, I.directed_path(4)),
              (3, I.chung_lu_digraph(2500, 6000, 2.2, 60, 0.2, rng)),
              (3, I.chung_lu_digraph(60, 150, 2.2, 20, 0.2, rng))]
    graphs = [ctx.load_graph(*g) for _, g in specs]
    try:
        alone = [ctx.count(g, ctx.table(k))[0] for (k, _), g in zip(specs, graphs)]
        srv = ctx.server(tick_units=32)
        try:
            tickets = [srv.submit(g, k) for (k, _), g in zip(specs, graphs)]
            res = [srv.wait(t, k)[0] for t, (k, _) in zip(tickets, specs)]
        finally:
            srv.stop()
        for h, a in zip(res, alone):
            assert np.array_equal(h, a)
        assert not res[4].any() and not res[5].any() and not res[6].any()
        assert_hist_equals_oracle(res[0], ctx.table(4).class_codes(), *specs[0][1], 4)
    finally:
        for g in graphs:
            g.free()


def test_served_graph_past_lds_limit(ctx):
    """A request whose graph is too large for LDS marks runs with marks in
    device memory inside the server too, beside a small one."""
    rng = np.random.default_rng(9100)
    big = I.er_digraph(M.MK_LDS_MARKS_MAX_VERTICES + 5000, 30000, rng)
    small = I.chung_lu_digraph(200, 600, 2.2, 30, 0.2, rng)
    gb, gs = ctx.load_graph(*big), ctx.load_graph(*small)
    try:
        alone = ctx.count(gb, ctx.table(4))[0]
        srv = ctx.server(tick_units=64)
        try:
            t1 = srv.submit(gb, 4)
            t2 = srv.submit(gs, 5)
            h1, _ = srv.wait(t1, 4)
            h2, _ = srv.wait(t2, 5)
        finally:
            srv.stop()
        assert np.array_equal(h1, alone)
        assert_hist_equals_oracle(h1, ctx.table(4).class_codes(), *big, 4)
        assert_hist_equals_oracle(h2, ctx.table(5).class_codes(), *small, 5)
    finally:
        gb.free()
        gs.free()


def test_admission_by_footprint(ctx):
    reqs = _requests(2, 6)
    graphs = [ctx.load_graph(*g) for _, g in reqs]
    biggest = max(g.footprint(k) for (k, _), g in zip(reqs, graphs))
    # budget for about one request at a time: all still complete, in order
    srv = ctx.server(hbm_budget_bytes=biggest + 1024, max_slots=2, tick_units=16)
    try:
        tickets = [srv.submit(g, k) for (k, _), g in zip(reqs, graphs)]
        res = [srv.wait(t, k) for t, (k, _) in zip(tickets, reqs)]
        for (hist, _), (k, _), g in zip(res, reqs, graphs):
            assert np.array_equal(hist, ctx.count(g, ctx.table(k))[0])
        with pytest.raises(M.MotifsError) as e:
            tiny = ctx.server(hbm_budget_bytes=1024)
            try:
                tiny.submit(graphs[0], reqs[0][0])
            finally:
                tiny.stop()
        assert e.value.status == M.MK_EBUSY
    finally:
        srv.stop()
        for g in graphs:
            g.free()


def test_timeout_and_unknown_ticket(ctx):
    big = ctx.load_graph(*I.k5_batch_graph(0))
    small = ctx.load_graph(*I.er_digraph(50, 150, np.random.default_rng(3)))
    ctx.table(5)
    srv = ctx.server(max_slots=1)
    try:
        t1 = srv.submit(big, 5)
        t2 = srv.submit(small, 3)
        # one slot: the second request stays queued behind the first
        with pytest.raises(M.MotifsError) as e:
            srv.wait(t2, 3, timeout_ms=0)
        assert e.value.status == M.MK_ETIMEDOUT
        h1, _ = srv.wait(t1, 5)
        h2, _ = srv.wait(t2, 3)
        assert h1.sum() > 0 and h2.sum() > 0
        with pytest.raises(M.MotifsError) as e:
            srv.wait(t2, 3, timeout_ms=0)
        assert e.value.status == M.MK_ENOTFOUND
        with pytest.raises(M.MotifsError) as e:
            srv.submit(small, 7)
        assert e.value.status == M.MK_ERANGE
    finally:
        srv.stop()
        big.free()
        small.free()
