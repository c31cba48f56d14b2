"""GPU class table (Section 3.2) against the oracle and closed forms."""

import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O

import combinatorics as C

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [3, 4, 5])
def test_table_entrywise_equals_oracle(ctx, k):
    t = ctx.table(k)
    canon, conn = O.canon_table(k)
    cc = O.class_codes(k)
    assert t.num_classes == len(cc)
    assert np.array_equal(t.class_codes(), cc)
    expect = np.where(conn.astype(bool), np.searchsorted(cc, canon), 0xFFFFFFFF).astype(np.uint32)
    got = t.read(0, 1 << (k * (k - 1)))
    assert np.array_equal(got, expect)
    assert t.lookup(int(cc[0])) == 0 and t.lookup((1 << (k * (k - 1))) - 1) == len(cc) - 1


def _aut_size(k, code):
    n = 0
    for p in itertools.permutations(range(k)):
        img = 0
        for i in range(k):
            for j in range(k):
                if i != j and (code >> O.bit_of(k, i, j)) & 1:
                    img |= 1 << O.bit_of(k, p[i], p[j])
        n += img == code
    return n


def test_table_k6(ctx):
    k = 6
    t = ctx.table(k)
    a = [1] + [C.unlabeled_digraphs(i) for i in range(1, 7)]
    assert t.num_classes == C.connected_from_all(a)[6] == 1530843
    cc = t.class_codes()
    assert np.all(np.diff(cc.astype(np.int64)) > 0)
    assert int(cc[0]) == (1 << (k - 1)) - 1 and int(cc[-1]) == (1 << 30) - 1
    # whole table in chunks: valid entries, per-class entry counts, self ids
    counts = np.zeros(t.num_classes, dtype=np.int64)
    valid = 0
    chunk = 1 << 26
    self_ids = np.full(t.num_classes, -1, dtype=np.int64)
    for first in range(0, 1 << 30, chunk):
        e = t.read(first, chunk)
        ok = e != 0xFFFFFFFF
        valid += int(ok.sum())
        assert int(e[ok].max(initial=0)) < t.num_classes
        counts += np.bincount(e[ok], minlength=t.num_classes)
        lo, hi = np.searchsorted(cc, [first, first + chunk])
        self_ids[lo:hi] = e[cc[lo:hi].astype(np.int64) - first]
    assert valid == C.labeled_connected_digraphs(6) == 1067308488
    assert np.array_equal(self_ids, np.arange(t.num_classes))
    assert np.all(720 % counts == 0)
    rng = np.random.default_rng(6)
    for cid in rng.choice(t.num_classes, size=40, replace=False).tolist() + [0, t.num_classes - 1]:
        code = int(cc[cid])
        assert O.canon(6, code) == code and O.connected(6, code)
        assert counts[cid] * _aut_size(6, code) == math.factorial(6)
    # random codes: the id of the oracle's canonical form, or invalid
    for code in rng.integers(0, 1 << 30, size=3000).tolist():
        got = t.lookup(int(code))
        if O.connected(6, code):
            c = O.canon(6, code)
            assert got == int(np.searchsorted(cc, c)) and cc[got] == c
        else:
            assert got == 0xFFFFFFFF


def test_table_errors(ctx):
    from paper_1804_09741_amd import motifs as M
    with pytest.raises(M.MotifsError) as e:
        ctx.table(7)
    assert e.value.status == M.MK_ERANGE
    t = ctx.table(3)
    with pytest.raises(M.MotifsError):
        t.lookup(64)
    with pytest.raises(M.MotifsError):
        t.class_code(13)
