"""Closed-form counts of directed graphs, computed without the oracle.

* unlabeled digraphs on k vertices: Burnside's lemma over S_k acting on the
  k(k-1) ordered vertex pairs (each permutation fixes 2^(#cycles) graphs);
* weakly connected unlabeled digraphs: inverse Euler transform of the above
  (a graph is a multiset of connected components);
* labeled weakly connected digraphs: exponential formula over the component
  holding vertex 1.
"""

import itertools
import math
from fractions import Fraction


def unlabeled_digraphs(k: int) -> int:
    pairs = [(i, j) for i in range(k) for j in range(k) if i != j]
    index = {p: t for t, p in enumerate(pairs)}
    total = 0
    for perm in itertools.permutations(range(k)):
        seen = [False] * len(pairs)
        cycles = 0
        for t in range(len(pairs)):
            if seen[t]:
                continue
            cycles += 1
            u = t
            while not seen[u]:
                seen[u] = True
                i, j = pairs[u]
                u = index[(perm[i], perm[j])]
        total += 2 ** cycles
    assert total % math.factorial(k) == 0
    return total // math.factorial(k)


def _mobius(n: int) -> int:
    res, p, m = 1, 2, n
    while p * p <= m:
        if m % p == 0:
            m //= p
            if m % p == 0:
                return 0
            res = -res
        p += 1
    if m > 1:
        res = -res
    return res


def connected_from_all(a):
    """Inverse Euler transform: a[0] = 1, a[n] = all graphs on n vertices ->
    c[n] = connected graphs on n vertices (n >= 1)."""
    N = len(a) - 1
    b = [0] * (N + 1)
    for n in range(1, N + 1):
        b[n] = n * a[n] - sum(b[j] * a[n - j] for j in range(1, n))
    c = [0] * (N + 1)
    for n in range(1, N + 1):
        s = sum(_mobius(n // d) * b[d] for d in range(1, n + 1) if n % d == 0)
        assert s % n == 0
        c[n] = s // n
    return c


def labeled_connected_digraphs(k: int) -> int:
    t = [2 ** (n * (n - 1)) for n in range(k + 1)]
    c = [0] * (k + 1)
    for n in range(1, k + 1):
        c[n] = t[n] - sum(math.comb(n - 1, j - 1) * c[j] * t[n - j] for j in range(1, n))
    return c[k]
