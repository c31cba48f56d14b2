"""Plausible mistakes planted in copies of the oracle (compiled with gcc on
the CPU) must each fail at least one pin: the pins are strong enough to
catch a wrong bit index, a dropped arc direction, a broken enumeration bound,
a transposed operand or an incomplete permutation walk."""

import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1804_09741_amd import inputs as I

import combinatorics as C

SRC = os.path.join(os.path.dirname(O.__file__), "oracle.c")

MUTANTS = {
    "bit index keeps the diagonal": (
        "return i * (k - 1) + j - (j > i ? 1 : 0);", "return i * (k - 1) + j - (j > i ? 0 : 0);"),
    "connectivity follows out-arcs only": (
        "if (!seen[w] && (a[u][w] || a[w][u])) {", "if (!seen[w] && (a[u][w])) {"),
    "canonical form is the maximum": (
        "if (c < best) best = c;", "if (c > best || best == 0xFFFFFFFFu) best = c;"),
    "permutation walk starts at the last relabeling": (
        "    for (int i = 0; i < k; ++i) p[i] = i;\n    uint32_t best",
        "    for (int i = 0; i < k; ++i) p[i] = k - 1 - i;\n    uint32_t best"),
    "extension ignores the root bound": (
        "if (u > root && !in_closed_nbhd(e, depth, u)) child[cn++] = u;",
        "if (u != root && !in_closed_nbhd(e, depth, u)) child[cn++] = u;"),
    "exclusive test drops one arc direction": (
        "if (s == u || arc(e, s, u) || arc(e, u, s)) return 1;",
        "if (s == u || arc(e, s, u)) return 1;"),
    "code operands transposed": (
        "if (i != j && arc(e, e->sub[i], e->sub[j])) code |= 1u << bit_of(k, i, j);",
        "if (i != j && arc(e, e->sub[j], e->sub[i])) code |= 1u << bit_of(k, i, j);"),
    "core test skips the second vertex": (
        "if (!y_touches || !z_touches) continue;", "if (!y_touches) continue;"),
    "core connectivity not checked": (
        "if (reached == nx) ++cores;", "++cores;"),
    "core pairs counted in both orders": (
        "for (int z = y + 1; z < k; ++z) {", "for (int z = 0; z < k; ++z) if (z != y) {"),
    "core touch follows out-arcs only": (
        "if (a[y][x[i]] || a[x[i]][y]) y_touches = 1;", "if (a[y][x[i]]) y_touches = 1;"),
    "switch allows loops": (
        "        if (a == d || c == b) continue;\n", ""),
    "switch skips the duplicate test": (
        "if (arc[(size_t)a * n + d] || arc[(size_t)c * n + b]) continue;", "if (0) continue;"),
    "generator mixing constant off by one": (
        "0xBF58476D1CE4E5B9ull", "0xBF58476D1CE4E5B8ull"),
    "child extension keeps the chosen vertex": (
        "for (int j = i + 1; j < next; ++j) child[cn++] = ext[j];",
        "for (int j = i; j < next; ++j) child[cn++] = ext[j];"),
    "k7 canonical form is the first relabeling": (
        "best = c < best ? c : best;", "best = best == ~0ull ? c : best;"),
    "k7 code operands transposed": (
        "if (i != j && arc7(e, e->sub[i], e->sub[j])) code |= 1ull << bit_of(7, i, j);",
        "if (i != j && arc7(e, e->sub[j], e->sub[i])) code |= 1ull << bit_of(7, i, j);"),
    "k7 exclusive test drops one arc direction": (
        "if (s == u || arc7(e, s, u) || arc7(e, u, s)) return 1;",
        "if (s == u || arc7(e, s, u)) return 1;"),
    "k7 extension ignores the root bound": (
        "if (u > root && !in_closed_nbhd7(e, depth, u)) child[cn++] = u;",
        "if (u != root && !in_closed_nbhd7(e, depth, u)) child[cn++] = u;"),
}


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path, name, text):
    src = tmp_path / (name + ".c")
    lib = tmp_path / (name + ".so")
    src.write_text(text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(src), "-o", str(lib)])
    return str(lib)


def _failed_pins_in_child(lib_path, timeout=120):
    """Run the pins against a library in a child process (a planted bug may
    loop forever; a timeout counts as caught)."""
    code = ("import sys, json; sys.path[:0] = %r; import test_oracle_mutants as T; "
            "from oracle import oracle as O; "
            "print(json.dumps(T._failed_pins(O.load_library(%r))))"
            % ([ROOT, os.path.join(ROOT, "tests")], lib_path))
    try:
        res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             timeout=timeout)
    except subprocess.TimeoutExpired:
        return ["timeout"]
    if res.returncode != 0:
        return ["crash: " + res.stderr[-300:]]
    return json.loads(res.stdout.strip().splitlines()[-1])


def _failed_pins(lib):
    """Names of the pins this oracle library fails."""
    failed = []
    tables = {}
    for k in (3, 4):
        canon, conn = O.canon_table_with(lib, k)
        tables[k] = canon
        cc = np.unique(canon[conn.astype(bool)])
        if len(cc) != {3: 13, 4: 199}[k]:
            failed.append("class count k=%d" % k)
        if len(np.unique(canon)) != C.unlabeled_digraphs(k):
            failed.append("burnside k=%d" % k)
        if int(conn.sum()) != C.labeled_connected_digraphs(k):
            failed.append("labeled connected k=%d" % k)
        if len(cc) and (int(cc[0]) != (1 << (k - 1)) - 1 or int(cc[-1]) != (1 << (k * (k - 1))) - 1):
            failed.append("extreme classes k=%d" % k)
    for k in (3, 4):
        try:
            star = O.count_with(lib, *I.out_star(7), k, tables[k])
            if star != {(1 << (k - 1)) - 1: math.comb(7, k - 1)}:
                failed.append("out-star k=%d" % k)
            rng = np.random.default_rng([55, k])
            for _ in range(3):
                g = I.er_digraph(8, int(rng.integers(8, 24)), rng)
                if O.count_with(lib, *g, k, tables[k]) != O.brute_force_count(*g, k):
                    failed.append("brute force k=%d" % k)
                    break
        except O.OracleError:
            failed.append("error k=%d" % k)
    # core multiplicity: closed forms, zero exactly on disconnected codes,
    # and the raw pair sums of tiny graphs
    try:
        for k in (3, 4, 5):
            full = (1 << (k * (k - 1))) - 1
            star = (1 << (k - 1)) - 1
            path = sum(1 << (i * (k - 1) + i) for i in range(k - 1))
            if (lib.oracle_core_mult(k, full) != math.comb(k, 2)
                    or lib.oracle_core_mult(k, star) != math.comb(k - 1, 2)
                    or lib.oracle_core_mult(k, path) != 1):
                failed.append("core closed forms k=%d" % k)
        for code in range(1 << 6):
            if (lib.oracle_core_mult(3, code) > 0) != bool(lib.oracle_connected(3, code)):
                failed.append("core zero iff disconnected")
                break
        rng = np.random.default_rng(56)
        for k in (3, 4):
            g = I.er_digraph(7, 14, rng)
            raw = O.core_pairs_count(*g, k)
            hist = O.brute_force_count(*g, k)
            if raw != {c: lib.oracle_core_mult(k, c) * v for c, v in hist.items()}:
                failed.append("core raw sums k=%d" % k)
    except O.OracleError:
        failed.append("core error")
    # k = 7: closed forms and the brute force on a tiny graph
    try:
        if O.count7_with(lib, *I.out_star(7)) != {63: 7}:
            failed.append("out-star k=7")
        if O.count7_with(lib, *I.complete_digraph(8)) != {(1 << 42) - 1: 8}:
            failed.append("complete digraph k=7")
        g = I.er_digraph(8, 16, np.random.default_rng(58))
        if O.count7_with(lib, *g) != O.brute_force_count(*g, 7):
            failed.append("brute force k=7")
    except O.OracleError:
        failed.append("error k=7")
    # ensemble: the generator's published values; switches keep the graph simple
    if [lib.oracle_splitmix64(0, i) for i in range(3)] != [
            0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f]:
        failed.append("splitmix64 values")
    rp, col = I.chung_lu_digraph(30, 90, 2.2, 10, 0.2, np.random.default_rng(57))
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    out = np.empty(len(col), dtype=np.int32)
    acc = lib.oracle_switch_chain(30, rp.ctypes.data, col.ctypes.data, 3, 0, 20 * len(col),
                                  200 * len(col), out.ctypes.data)
    arcs = {(u, int(out[t])) for u in range(30) for t in range(rp[u], rp[u + 1])}
    if acc < 0 or len(arcs) != len(col) or any(u == v for u, v in arcs):
        failed.append("switch simplicity")
    return failed


def test_unmutated_oracle_passes(tmp_path):
    lib = _build(tmp_path, "clean", open(SRC).read())
    assert _failed_pins_in_child(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    before, after = MUTANTS[name]
    text = open(SRC).read()
    # the first site: a k = 7 copy of a line further down keeps its own mutant
    assert text.count(before) >= 1, "mutation site not found: %s" % before
    lib = _build(tmp_path, "mutant", text.replace(before, after, 1))
    assert _failed_pins_in_child(lib), "no pin catches: %s" % name
