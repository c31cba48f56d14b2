"""The pruning rule of the GPU's k = 7 canonical form, modelled on the CPU
and checked against the brute-force minimum over all 5,040 relabelings (no
GPU).  Rule: the minimum code has at position 6 a vertex of the least
out-degree d and its out-neighbours at positions 0..d-1; when d = 0, at
position 5 a vertex without an arc to position 6 if one exists, of the
least out-degree towards the other five among those, and its
out-neighbours at 0..d5-1.  The code's bit for arc i -> j is
6 i + j - [j > i] (row-major adjacency matrix without its diagonal)."""

import itertools
import random


def _bit(i, j):
    return 6 * i + j - (1 if j > i else 0)


def _arcs(code):
    out = []
    for b in range(42):
        if code >> b & 1:
            i, r = divmod(b, 6)
            out.append((i, r + (1 if r >= i else 0)))
    return out


def _relabel(code, sigma):
    c = 0
    for i, j in _arcs(code):
        c |= 1 << _bit(sigma[i], sigma[j])
    return c


def _brute(code):
    return min(_relabel(code, p) for p in itertools.permutations(range(7)))


def _out(code, v):
    return {j for i, j in _arcs(code) if i == v}


def _pruned(code):
    """Minimum over the relabelings the rule keeps, and their number."""
    od = [len(_out(code, v)) for v in range(7)]
    d6 = min(od)
    best, tried = None, 0
    for c6 in [v for v in range(7) if od[v] == d6]:
        groups = []
        if d6 > 0:
            on = sorted(_out(code, c6))
            groups = [(c6, 6, on, [v for v in range(7) if v != c6 and v not in on])]
        else:
            keys = {v: (c6 in _out(code, v), len(_out(code, v) - {c6}))
                    for v in range(7) if v != c6}
            kmin = min(keys.values())
            for c5 in [v for v in keys if keys[v] == kmin]:
                on = sorted(_out(code, c5) - {c6})
                groups.append((c6, 6, on, [v for v in range(7) if v not in (c6, c5) and v not in on],
                               c5))
        for g in groups:
            for pn in itertools.permutations(g[2]):
                for pr in itertools.permutations(g[3]):
                    sigma = [0] * 7
                    sigma[g[0]] = 6
                    if len(g) == 5:
                        sigma[g[4]] = 5
                    for pos, v in enumerate(pn):
                        sigma[v] = pos
                    for pos, v in enumerate(pr):
                        sigma[v] = len(pn) + pos
                    assert sorted(sigma) == list(range(7))
                    c = _relabel(code, sigma)
                    tried += 1
                    best = c if best is None or c < best else best
    return best, tried


def _connected(nar, rng):
    while True:
        es = set()
        while len(es) < nar:
            i, j = rng.sample(range(7), 2)
            es.add((i, j))
        adj = {v: set() for v in range(7)}
        for i, j in es:
            adj[i].add(j)
            adj[j].add(i)
        seen, st = {0}, [0]
        while st:
            x = st.pop()
            for y in adj[x] - seen:
                seen.add(y)
                st.append(y)
        if len(seen) == 7:
            return sum(1 << _bit(i, j) for i, j in es)


def test_rule_reaches_the_minimum():
    rng = random.Random(70)
    codes = [_connected(rng.choice([6, 7, 8, 10, 14]), rng) for _ in range(40)]
    codes += [sum(1 << b for b in range(42) if rng.random() < 0.5) for _ in range(8)]
    codes += [sum(1 << _bit(0, j) for j in range(1, 7)),        # out-star
              sum(1 << _bit(j, 0) for j in range(1, 7)),        # in-star
              sum(1 << _bit(i, (i + 1) % 7) for i in range(7)),  # directed cycle
              (1 << 42) - 1, 0]
    tried = 0
    for c in codes:
        p, n = _pruned(c)
        assert p == _brute(c), c
        tried += n
    assert tried < 5040 * len(codes) / 3
