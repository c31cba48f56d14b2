"""Digests of histograms and graphs for the stored oracle results.

A histogram is written as its (canonical code, count) pairs with count > 0,
ascending by code, each pair two little-endian uint64; its digest is the
first 32 hex digits of the SHA-256 of those bytes.  A graph's digest covers
its CSR arrays (little-endian int32), so a change in the seeded generators
shows up as a changed input, not as a parity failure.  No method arithmetic
here: both the GPU histograms and the oracle's go through the same
serialisation.
"""

import hashlib

import numpy as np


def pairs_digest(codes, counts) -> str:
    codes = np.asarray(codes, dtype=np.uint64)
    counts = np.asarray(counts, dtype=np.uint64)
    keep = counts > 0
    codes, counts = codes[keep], counts[keep]
    order = np.argsort(codes, kind="stable")
    a = np.stack([codes[order], counts[order]], axis=1).astype("<u8")
    return hashlib.sha256(a.tobytes()).hexdigest()[:32]


def dict_digest(h) -> str:
    """Digest of {canonical code: count}."""
    keys = sorted(h)
    return pairs_digest(keys, [h[c] for c in keys])


def dense_digest(hist, class_codes) -> str:
    """Digest of a dense histogram indexed by class id."""
    hist = np.asarray(hist, dtype=np.uint64)
    nz = np.flatnonzero(hist)
    return pairs_digest(np.asarray(class_codes)[nz], hist[nz])


def graph_digest(row_ptr, col) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(row_ptr, dtype="<i4").tobytes())
    h.update(b"|")
    h.update(np.ascontiguousarray(col, dtype="<i4").tobytes())
    return h.hexdigest()[:32]
