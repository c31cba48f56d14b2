"""The C-ABI library loads and exports every symbol include/motifs.h
declares; the Python binding covers exactly those (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_1804_09741_amd import motifs as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    """Every function the headers under include/ declare."""
    names = set()
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            with open(os.path.join(ROOT, "include", name)) as f:
                hdr = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
            names |= set(re.findall(r"\b(mk_\w+)\s*\(", hdr))
    return names


def _lib():
    if not os.path.exists(M.LIB_PATH):
        pytest.skip("libmotifs.so not built")
    return ctypes.CDLL(M.LIB_PATH)


def test_every_declared_symbol_is_exported():
    lib = _lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_matches_header():
    assert set(M.SIGNATURES) == _declared()


def test_status_strings():
    lib = M.library()
    for code in (M.MK_OK, M.MK_EINVAL, M.MK_ERANGE, M.MK_EGRAPH, M.MK_ENOMEM, M.MK_EDEVICE,
                 M.MK_EBUSY, M.MK_ETIMEDOUT, M.MK_ENOTFOUND):
        s = lib.mk_status_str(code).decode()
        assert s and s != "unknown status"
    assert lib.mk_status_str(-99).decode() == "unknown status"


def test_null_arguments_rejected_without_device():
    lib = M.library()
    assert lib.mk_init(0, None) == M.MK_EINVAL
    assert lib.mk_graph_info(None, None, None, None) == M.MK_EINVAL
    assert lib.mk_table_info(None, None, None, None, None) == M.MK_EINVAL
    assert lib.mk_batch_stats_get(None, None) == M.MK_EINVAL
    assert lib.mk_server_stop(None) == M.MK_EINVAL
    assert b"NULL" in lib.mk_last_error()


def test_constants_match_header():
    with open(os.path.join(ROOT, "include", "motifs.h")) as f:
        hdr = f.read()
    for name in ("MK_OK", "MK_EINVAL", "MK_ERANGE", "MK_EGRAPH", "MK_ENOMEM", "MK_EDEVICE",
                 "MK_EBUSY", "MK_ETIMEDOUT", "MK_ENOTFOUND", "MK_MAX_VERTICES", "MK_MAX_DEGREE",
                 "MK_LDS_MARKS_MAX_VERTICES"):
        m = re.search(r"#define %s (\(?-?\d+(?: << \d+)?\)?)\s" % name, hdr)
        assert m, name
        expr = m.group(1).strip("()")
        value = (int(expr.split("<<")[0]) << int(expr.split("<<")[1])) if "<<" in expr else int(expr)
        assert value == getattr(M, name), name
    for prefix, names in (("MK_METHOD_", ("AUTO", "ESU", "CORES")),
                          ("MK_ADJ_", ("AUTO", "BITS", "LISTS")),
                          ("MK_MARKS_", ("AUTO", "LDS", "GLOBAL"))):
        for name in names:
            m = re.search(r"#define %s%s (\d+)" % (prefix, name), hdr)
            assert m and int(m.group(1)) == getattr(M, prefix[3:] + name), prefix + name
