"""Seeded synthetic directed graphs for the Motifs-k workloads.

This module only draws graphs.  It holds none of the counting method's
arithmetic (no enumeration, no adjacency codes, no classes), so both the
GPU path and the CPU oracle can be fed from it without sharing any of
the method.

Every graph is a simple digraph: no self-loops and no repeated arcs.  A
pair of opposite arcs (u, v), (v, u) is a bidirected edge of the paper
(Section 2, notation) and counts as two arcs in ``m``.

Graphs are returned as an out-adjacency CSR pair ``(row_ptr, col)`` of
int32 numpy arrays, rows sorted, which is what the library's graph
loader takes.

The paper's eight datasets (Table "Summary of the data sets") are not
available, so these recipes stand in for them: sparse, hub-heavy
digraphs with n and m in the same ranges (n 100..7000, m up to ~30000).
"""

from __future__ import annotations

import dataclasses
import functools
from typing import List, Tuple

import numpy as np

Csr = Tuple[np.ndarray, np.ndarray]


# --------------------------------------------------------------------------
# basic conversions
# --------------------------------------------------------------------------

def csr_from_arcs(n: int, src, dst) -> Csr:
    """Out-adjacency CSR of the arcs ``src[i] -> dst[i]`` (rows sorted)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr.astype(np.int32), dst.astype(np.int32)


def arcs_from_csr(row_ptr, col) -> Tuple[np.ndarray, np.ndarray]:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    return src, np.asarray(col, dtype=np.int64)


def relabel(row_ptr, col, perm) -> Csr:
    """The same digraph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src, dst = arcs_from_csr(row_ptr, col)
    return csr_from_arcs(len(perm), perm[src], perm[dst])


def reverse(row_ptr, col) -> Csr:
    """The digraph with every arc turned around."""
    src, dst = arcs_from_csr(row_ptr, col)
    return csr_from_arcs(len(row_ptr) - 1, dst, src)


def disjoint_union(graphs) -> Csr:
    srcs, dsts, off = [], [], 0
    for rp, cl in graphs:
        s, d = arcs_from_csr(rp, cl)
        srcs.append(s + off)
        dsts.append(d + off)
        off += len(rp) - 1
    return csr_from_arcs(off, np.concatenate(srcs) if srcs else [],
                         np.concatenate(dsts) if dsts else [])


# --------------------------------------------------------------------------
# small fixed families (closed-form test graphs)
# --------------------------------------------------------------------------

def complete_digraph(n: int) -> Csr:
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = s != d
    return csr_from_arcs(n, s[mask], d[mask])


def out_star(leaves: int) -> Csr:
    return csr_from_arcs(leaves + 1, np.zeros(leaves), np.arange(1, leaves + 1))


def in_star(leaves: int) -> Csr:
    return csr_from_arcs(leaves + 1, np.arange(1, leaves + 1), np.zeros(leaves))


def directed_cycle(n: int) -> Csr:
    v = np.arange(n)
    return csr_from_arcs(n, v, (v + 1) % n)


def bidirected_cycle(n: int) -> Csr:
    v = np.arange(n)
    return csr_from_arcs(n, np.concatenate([v, (v + 1) % n]),
                         np.concatenate([(v + 1) % n, v]))


def directed_path(n: int) -> Csr:
    v = np.arange(n - 1)
    return csr_from_arcs(n, v, v + 1)


def empty_graph(n: int) -> Csr:
    return csr_from_arcs(n, [], [])


# --------------------------------------------------------------------------
# random families
# --------------------------------------------------------------------------

def _first_occurrence(keys: np.ndarray) -> np.ndarray:
    """Indices of the first occurrence of each key, in original order."""
    _, first = np.unique(keys, return_index=True)
    first.sort()
    return first


def _occurrence_rank(values: np.ndarray) -> np.ndarray:
    """r[i] = number of j < i with values[j] == values[i]."""
    order = np.argsort(values, kind="stable")
    sv = values[order]
    starts = np.r_[0, np.flatnonzero(sv[1:] != sv[:-1]) + 1]
    run_id = np.cumsum(np.r_[0, (sv[1:] != sv[:-1]).astype(np.int64)])
    rank_sorted = np.arange(len(sv)) - starts[run_id]
    rank = np.empty_like(rank_sorted)
    rank[order] = rank_sorted
    return rank


def _sample_arcs(n, target, p_out, p_in, rng, cap_out=None, cap_in=None):
    """Draw arcs u~p_out, v~p_in until `target` distinct non-loop arcs.

    Arcs that would repeat an arc, close a loop, or push an out-degree past
    cap_out (in-degree past cap_in) are rejected.
    """
    keys = np.zeros(0, dtype=np.int64)
    outdeg = np.zeros(n, dtype=np.int64)
    indeg = np.zeros(n, dtype=np.int64)
    big = np.iinfo(np.int64).max
    cap_out = big if cap_out is None else cap_out
    cap_in = big if cap_in is None else cap_in
    rounds = 0
    while len(keys) < target:
        rounds += 1
        if rounds > 10000:
            raise RuntimeError("arc sampler made no progress (caps too tight?)")
        need = target - len(keys)
        batch = max(2 * need, 1024)
        u = rng.choice(n, size=batch, p=p_out)
        v = rng.choice(n, size=batch, p=p_in)
        ok = u != v
        u, v = u[ok], v[ok]
        k = u * n + v
        first = _first_occurrence(k)
        u, v, k = u[first], v[first], k[first]
        fresh = ~np.isin(k, keys)
        u, v, k = u[fresh], v[fresh], k[fresh]
        ok = (outdeg[u] + _occurrence_rank(u) < cap_out) & \
             (indeg[v] + _occurrence_rank(v) < cap_in)
        u, v, k = u[ok][:need], v[ok][:need], k[ok][:need]
        np.add.at(outdeg, u, 1)
        np.add.at(indeg, v, 1)
        keys = np.concatenate([keys, k])
    return keys // n, keys % n


def er_digraph(n: int, m: int, rng) -> Csr:
    """Directed G(n, m): m distinct non-loop arcs drawn uniformly."""
    if m > n * (n - 1):
        raise ValueError("m exceeds n(n-1)")
    p = np.full(n, 1.0 / n)
    s, d = _sample_arcs(n, m, p, p, rng)
    return csr_from_arcs(n, s, d)


def _capped_weights(n, gamma, total, cap, rng):
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w = rng.permutation(w)
    for _ in range(200):
        w = w * (total / w.sum())
        if cap is None or w.max() <= cap * (1 + 1e-12):
            break
        w = np.minimum(w, cap)
    return w


def chung_lu_digraph(n: int, m: int, gamma: float, cap, reciprocity: float,
                     rng) -> Csr:
    """Directed Chung-Lu graph with power-law expected in/out degrees.

    Expected out- and in-degree sequences are w_i ~ i^(-1/(gamma-1)),
    independently permuted (uncorrelated), rescaled to the base arc count
    m_b = round(m / (1 + reciprocity)) and capped at ``cap``.  Base arcs are
    drawn with u ~ w_out and v ~ w_in; realised out/in-degrees never exceed
    ``cap``.  Then reverses of uniformly chosen arcs that lack one are added
    until there are m arcs.
    """
    m_b = int(round(m / (1.0 + reciprocity)))
    w_out = _capped_weights(n, gamma, m_b, cap, rng)
    w_in = _capped_weights(n, gamma, m_b, cap, rng)
    s, d = _sample_arcs(n, m_b, w_out / w_out.sum(), w_in / w_in.sum(), rng,
                        cap_out=cap, cap_in=cap)
    extra = m - m_b
    if extra > 0:
        keys = set((s * n + d).tolist())
        outdeg = np.bincount(s, minlength=n)
        indeg = np.bincount(d, minlength=n)
        order = rng.permutation(len(s))
        add_s, add_d = [], []
        big = np.iinfo(np.int64).max if cap is None else cap
        for i in order:
            a, b = int(s[i]), int(d[i])
            if b * n + a in keys:
                continue
            if outdeg[b] >= big or indeg[a] >= big:
                continue
            keys.add(b * n + a)
            outdeg[b] += 1
            indeg[a] += 1
            add_s.append(b)
            add_d.append(a)
            if len(add_s) == extra:
                break
        s = np.concatenate([s, np.asarray(add_s, dtype=np.int64)])
        d = np.concatenate([d, np.asarray(add_d, dtype=np.int64)])
    return csr_from_arcs(n, s, d)


def powerlaw_out_digraph(n: int, m: int, exponent: float, dmax: int,
                         rng) -> Csr:
    """Out-degrees i.i.d. P(d) ~ d^-exponent on [1, dmax], adjusted by +-1 at
    random vertices (staying in [0, dmax]) to sum exactly m; each vertex's
    targets are drawn uniformly without replacement from the other vertices,
    so in-degrees are close to Poisson."""
    ds = np.arange(1, dmax + 1, dtype=np.float64)
    p = ds ** (-exponent)
    p /= p.sum()
    deg = rng.choice(np.arange(1, dmax + 1), size=n, p=p).astype(np.int64)
    while deg.sum() != m:
        v = int(rng.integers(n))
        if deg.sum() < m and deg[v] < min(dmax, n - 1):
            deg[v] += 1
        elif deg.sum() > m and deg[v] > 0:
            deg[v] -= 1
    src, dst = [], []
    for u in range(n):
        if deg[u] == 0:
            continue
        t = rng.choice(n - 1, size=int(deg[u]), replace=False)
        t = t + (t >= u)
        src.append(np.full(len(t), u))
        dst.append(t)
    return csr_from_arcs(n, np.concatenate(src), np.concatenate(dst))


def sparse_powerlaw_digraph(n: int, exponent: float, dmax: int, rng) -> Csr:
    """Large sparse graphs drawn in vectorised form: out-degrees i.i.d.
    P(d) ~ d^-exponent on [1, dmax]; targets uniform over the other vertices,
    a repeated target dropped (so m is about n times the mean out-degree);
    in-degrees close to Poisson."""
    ds = np.arange(1, dmax + 1, dtype=np.float64)
    p = ds ** (-exponent)
    p /= p.sum()
    deg = rng.choice(np.arange(1, dmax + 1), size=n, p=p).astype(np.int64)
    deg = np.minimum(deg, n - 1)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    t = rng.integers(0, n - 1, size=len(src))
    dst = t + (t >= src)
    keep = _first_occurrence(src * n + dst)
    return csr_from_arcs(n, src[keep], dst[keep])


def switch_randomise(row_ptr, col, accepted: int, rng) -> Csr:
    """Degree-preserving randomisation by directed arc switches.

    Repeatedly pick two arcs a->b, c->d uniformly and replace them by a->d,
    c->b unless that would make a loop or repeat an arc (or the switch is a
    no-op).  Stops after ``accepted`` switches.  Every vertex keeps its out-
    and in-degree exactly.
    """
    n = len(row_ptr) - 1
    s, d = arcs_from_csr(row_ptr, col)
    s, d = s.copy(), d.copy()
    m = len(s)
    if m < 2 or accepted == 0:
        return csr_from_arcs(n, s, d)
    keys = set((s * n + d).tolist())
    done, tries = 0, 0
    limit = 200 * accepted + 10000
    while done < accepted:
        picks = rng.integers(0, m, size=(4096, 2))
        for i, j in picks.tolist():
            tries += 1
            if tries > limit:
                raise RuntimeError("switch randomisation stalled")
            a, b, c, e = s[i], d[i], s[j], d[j]
            if a == c or b == e or a == e or c == b:
                continue
            k1, k2 = a * n + e, c * n + b
            if k1 in keys or k2 in keys:
                continue
            keys.discard(a * n + b)
            keys.discard(c * n + e)
            keys.add(k1)
            keys.add(k2)
            d[i], d[j] = e, b
            done += 1
            if done == accepted:
                break
    return csr_from_arcs(n, s, d)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    k: int
    graphs: Tuple[Csr, ...]


def _rng(cfg: int, idx: int):
    return np.random.default_rng([cfg, idx])


@functools.lru_cache(maxsize=None)
def workload_k3_er() -> Workload:
    """k=3, one directed G(n=200, m=800)."""
    g = er_digraph(200, 800, _rng(1, 0))
    return Workload("k3_er_n200_m800", 3, (g,))


@functools.lru_cache(maxsize=None)
def workload_k4_chunglu() -> Workload:
    """k=4, one directed Chung-Lu graph n=2000, m=10000, gamma=2.2,
    cap 200, 20% reciprocal."""
    g = chung_lu_digraph(2000, 10000, 2.2, 200, 0.2, _rng(2, 0))
    return Workload("k4_chunglu_n2000_m10000", 4, (g,))


@functools.lru_cache(maxsize=None)
def _k5_original():
    return chung_lu_digraph(1000, 3000, 2.1, 200, 0.1, _rng(3, 0))


@functools.lru_cache(maxsize=None)
def k5_batch_graph(idx: int) -> Csr:
    """Graph idx of the k=5 batch: 0 = original, r = r-th randomisation."""
    g = _k5_original()
    if idx == 0:
        return g
    return switch_randomise(*g, accepted=10 * 3000, rng=_rng(3, idx))


def workload_k5_batch(count: int = 101) -> Workload:
    """k=5: original Chung-Lu n=1000, m=3000, gamma=2.1, 10% reciprocal,
    plus 100 degree-preserving randomisations (10*m accepted switches)."""
    gs = tuple(k5_batch_graph(i) for i in range(count))
    return Workload("k5_batch%d_chunglu_n1000_m3000" % count, 5, gs)


@functools.lru_cache(maxsize=None)
def _k6_original():
    return powerlaw_out_digraph(700, 1500, 2.5, 60, _rng(4, 0))


@functools.lru_cache(maxsize=None)
def k6_batch_graph(idx: int) -> Csr:
    g = _k6_original()
    if idx == 0:
        return g
    return switch_randomise(*g, accepted=10 * 1500, rng=_rng(4, idx))


def workload_k6_batch(count: int = 31) -> Workload:
    """k=6: original power-law out-degree graph n=700, m=1500 (exponent 2.5,
    out-degree <= 60, in-degree ~Poisson) plus 30 randomisations."""
    gs = tuple(k6_batch_graph(i) for i in range(count))
    return Workload("k6_batch%d_powerlaw_n700_m1500" % count, 6, gs)


def workload_k6_large(n: int = 1 << 20) -> Workload:
    """k=6 on one graph past the LDS marks limit: the k=6 batch's degree
    recipe (out-degree P(d) ~ d^-2.5 on [1, 60], uniform targets) at
    n = 2^20 vertices (m ~ 2.2 n)."""
    g = sparse_powerlaw_digraph(n, 2.5, 60, _rng(6, 0))
    return Workload("k6_large_powerlaw_n%d_m%d" % (n, len(g[1])), 6, (g,))


@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    k: int
    graph: Csr


def serving_request(i: int, seed: int = 5, n_max: int = 5000) -> Tuple[int, Csr]:
    """(k, graph) of request i of the stream: k ~ U{3..6}, n ~ U[100, n_max],
    m = round(n*U[2,6]), gamma ~ U[2.0, 2.6], no reciprocity, degrees capped
    at 200 for k<=5 and 60 for k=6 (so that every request has a bounded
    number of k-subgraphs).  Request i depends only on (seed, i)."""
    r = np.random.default_rng([5, seed, i])
    k = int(r.integers(3, 7))
    n = int(r.integers(100, n_max + 1))
    m = int(round(n * r.uniform(2.0, 6.0)))
    gamma = float(r.uniform(2.0, 2.6))
    cap = 200 if k <= 5 else 60
    return k, chung_lu_digraph(n, m, gamma, cap, 0.0, r)


def serving_arrivals(count: int = 1000, rate_per_s: float = 100.0, seed: int = 5) -> np.ndarray:
    """Poisson arrival times (seconds, the first at 0) of the stream."""
    rng = np.random.default_rng([5, seed])
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps) - gaps[0]


def serving_requests(count: int = 1000, rate_per_s: float = 100.0,
                     seed: int = 5, n_max: int = 5000) -> List[Request]:
    """The first ``count`` requests of the stream (``serving_request``) with
    Poisson arrivals at ``rate_per_s``."""
    t = serving_arrivals(count, rate_per_s, seed)
    out = []
    for i in range(count):
        k, g = serving_request(i, seed, n_max)
        out.append(Request(float(t[i]), k, g))
    return out


def check_simple(row_ptr, col) -> None:
    """Raise ValueError unless (row_ptr, col) is a simple digraph CSR."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    n = len(row_ptr) - 1
    if n < 0 or row_ptr[0] != 0 or np.any(np.diff(row_ptr) < 0) \
            or row_ptr[-1] != len(col):
        raise ValueError("bad row_ptr")
    if len(col) and (col.min() < 0 or col.max() >= n):
        raise ValueError("vertex id out of range")
    s, d = arcs_from_csr(row_ptr, col)
    if np.any(s == d):
        raise ValueError("self-loop")
    if len(np.unique(s * max(n, 1) + d)) != len(s):
        raise ValueError("repeated arc")
