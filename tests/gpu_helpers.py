"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

import numpy as np

from oracle import oracle as O


def as_code_dict(hist, class_codes):
    """Dense GPU histogram -> {canonical code: count} (zeros dropped)."""
    nz = np.flatnonzero(hist)
    return {int(class_codes[i]): int(hist[i]) for i in nz}


def assert_hist_equals_oracle(hist, class_codes, row_ptr, col, k):
    """Bit-exact comparison with the CPU oracle through canonical codes."""
    got = as_code_dict(hist, class_codes)
    exp = O.count(row_ptr, col, k)
    assert got == exp, _diff(got, exp)


def _diff(got, exp):
    keys = sorted(set(got) | set(exp))
    bad = [(c, got.get(c, 0), exp.get(c, 0)) for c in keys if got.get(c, 0) != exp.get(c, 0)]
    return "%d classes differ, first: %s; totals gpu=%d oracle=%d" % (
        len(bad), bad[:5], sum(got.values()), sum(exp.values()))
