"""Python binding of libmotifs.so (the C ABI in include/motifs.h).

Argument marshalling only: every step of the Motifs-k path runs in the HIP
library.  The module-level functions carry the C names (``mk_init``,
``mk_graph_load_csr``, ``mk_table_build``, ``mk_count``, ...) and raise
:class:`MotifsError` on a negative status; the small classes at the bottom
wrap the handles.  Device buffers for ``mk_batch_run`` may be torch tensors
(PyTorch supplies device memory and streams, nothing else).

The library must have been built (``python -m paper_1804_09741_amd.build``);
there is no fallback of any kind.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmotifs.so")

MK_OK = 0
MK_EINVAL = -1
MK_ERANGE = -2
MK_EGRAPH = -3
MK_ENOMEM = -4
MK_EDEVICE = -5
MK_EBUSY = -6
MK_ETIMEDOUT = -7
MK_ENOTFOUND = -8
MK_INVALID_CLASS = 0xFFFFFFFF
MK_MAX_VERTICES = 1 << 20
MK_MAX_DEGREE = 4096
MK_LDS_MARKS_MAX_VERTICES = 8192

NUM_CLASSES = {3: 13, 4: 199, 5: 9364, 6: 1530843}


class MotifsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d): %s" % (_status_name(status), status, message))
        self.status = status


class BatchOpts(ctypes.Structure):
    _fields_ = [("split_threshold", ctypes.c_uint64), ("waves_per_cu", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("units_per_grab", ctypes.c_int32),
                ("units_per_wave", ctypes.c_int32), ("method", ctypes.c_int32),
                ("adjacency", ctypes.c_int32), ("marks", ctypes.c_int32)]


METHOD_AUTO, METHOD_ESU, METHOD_CORES = 0, 1, 2
ADJ_AUTO, ADJ_BITS, ADJ_LISTS = 0, 1, 2
MARKS_AUTO, MARKS_LDS, MARKS_GLOBAL = 0, 1, 2


class BatchStats(ctypes.Structure):
    _fields_ = [("units", ctypes.c_uint64), ("split_pairs", ctypes.c_uint64),
                ("grid", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("k", ctypes.c_int32), ("ng", ctypes.c_int32), ("method", ctypes.c_int32),
                ("adjacency", ctypes.c_int32), ("marks", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("tick_units", ctypes.c_int32)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submit_us", ctypes.c_double), ("admit_us", ctypes.c_double),
                ("done_us", ctypes.c_double)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_I64 = ctypes.c_int64

# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "mk_init": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "mk_destroy": (None, [_P]),
    "mk_device_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I64)]),
    "mk_graph_load_csr": (ctypes.c_int, [_P, _I32, _P, _P, ctypes.POINTER(_P)]),
    "mk_graph_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                                     ctypes.POINTER(_I32)]),
    "mk_graph_footprint": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_U64)]),
    "mk_graph_free": (None, [_P]),
    "mk_graph_read": (ctypes.c_int, [_P, _P, _P]),
    "mk_randomise": (ctypes.c_int, [_P, _P, _I32, _U64, _U32, _P, _P]),
    "mk_significance": (ctypes.c_int, [_P, _P, _I32, _U32, _P, _P]),
    "mk_table_build": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(_P)]),
    "mk_table_release": (ctypes.c_int, [_P, ctypes.c_int]),
    "mk_table_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_U32),
                                     ctypes.POINTER(_U64), ctypes.POINTER(ctypes.c_double)]),
    "mk_table_class_code": (ctypes.c_int, [_P, _U32, ctypes.POINTER(_U32)]),
    "mk_table_class_codes": (ctypes.c_int, [_P, _P, _U32]),
    "mk_table_lookup": (ctypes.c_int, [_P, _U32, ctypes.POINTER(_U32)]),
    "mk_table_read": (ctypes.c_int, [_P, _U64, _U64, _P]),
    "mk_table_core_mult": (ctypes.c_int, [_P, _U32, _U32, _P]),
    "mk_count": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(_U64)]),
    "mk_count_batch": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P]),
    "mk_count_static": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "mk_static_scratch_bytes": (_U64, []),
    "mk_count7": (ctypes.c_int, [_P, _P, _I32, _I64, _P, _P, _P, _P,
                                 ctypes.POINTER(ctypes.c_double)]),
    "mk_batch_create": (ctypes.c_int, [_P, _P, _I32, _P, ctypes.POINTER(BatchOpts),
                                       ctypes.POINTER(_P)]),
    "mk_batch_run": (ctypes.c_int, [_P, _P, _P]),
    "mk_batch_read": (ctypes.c_int, [_P, _P, _P]),
    "mk_batch_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(BatchStats)]),
    "mk_batch_timing": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
    "mk_batch_free": (None, [_P]),
    "mk_k7_cache_info": (ctypes.c_int, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "mk_k7_cache_clear": (ctypes.c_int, [_P]),
    "mk_autotune": (ctypes.c_int, [_P, _P, _I32, _P, _I32, ctypes.POINTER(BatchOpts),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]),
    "mk_batch_debug": (ctypes.c_int, [_P, _I32]),
    "mk_server_start": (ctypes.c_int, [_P, ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    "mk_submit": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.POINTER(_U64)]),
    "mk_wait": (ctypes.c_int, [_P, _U64, _P, _U32, _I32, ctypes.POINTER(RequestTimes)]),
    "mk_server_stop": (ctypes.c_int, [_P]),
    "mk_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "mk_last_error": (ctypes.c_char_p, []),
}

_lib = None


def library() -> ctypes.CDLL:
    """The loaded libmotifs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmotifs.so is not built (%s); run "
                               "`python -m paper_1804_09741_amd.build`" % LIB_PATH)
        # PyTorch ships its own HIP runtime with the same soname as ROCm's;
        # whichever loads first serves the process.  Load torch's first so
        # that torch tensors/streams and this library share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name, None)
            if fn is None:  # reported by the symbol test; calls raise AttributeError
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_name(status: int) -> str:
    try:
        return library().mk_status_str(status).decode()
    except Exception:  # library not loadable: plain number
        return "status"


def _check(rc: int) -> int:
    if rc < 0:
        raise MotifsError(rc, library().mk_last_error().decode())
    return rc


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P) if a.size else None


# ------------------------------------------------------------------ context

def mk_init(device: int = 0) -> int:
    h = _P()
    _check(library().mk_init(device, ctypes.byref(h)))
    return h.value


def mk_destroy(ctx: int) -> None:
    library().mk_destroy(ctx)


def mk_device_info(ctx: int) -> Tuple[int, int]:
    cu, mem = _I32(), _I64()
    _check(library().mk_device_info(ctx, ctypes.byref(cu), ctypes.byref(mem)))
    return cu.value, mem.value


# -------------------------------------------------------------------- graph

def mk_graph_load_csr(ctx: int, row_ptr, col) -> int:
    row_ptr = _i32(row_ptr)
    col = _i32(col)
    n = len(row_ptr) - 1
    if n < 0:
        raise MotifsError(MK_EINVAL, "row_ptr must have n+1 >= 1 entries")
    if len(col) < int(row_ptr[-1]):
        raise MotifsError(MK_EINVAL, "col shorter than row_ptr[n]")
    h = _P()
    _check(library().mk_graph_load_csr(ctx, n, row_ptr.ctypes.data_as(_P), _ptr(col),
                                       ctypes.byref(h)))
    return h.value


def mk_graph_info(g: int) -> Tuple[int, int, int]:
    n, m, d = _I32(), _I64(), _I32()
    _check(library().mk_graph_info(g, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d)))
    return n.value, m.value, d.value


def mk_graph_footprint(g: int, k: int) -> int:
    b = _U64()
    _check(library().mk_graph_footprint(g, k, ctypes.byref(b)))
    return b.value


def mk_graph_read(g: int) -> Tuple[np.ndarray, np.ndarray]:
    n, m, _ = mk_graph_info(g)
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(m, 1), dtype=np.int32)
    _check(library().mk_graph_read(g, row_ptr.ctypes.data_as(_P), col.ctypes.data_as(_P)))
    return row_ptr, col[:m]


def mk_randomise(ctx: int, g: int, count: int, seed: int,
                 switches_per_arc: int) -> Tuple[list, np.ndarray]:
    """(handles of `count` random graphs, accepted switches per graph)."""
    hs = (_P * max(count, 1))()
    acc = np.zeros(max(count, 1), dtype=np.uint64)
    _check(library().mk_randomise(ctx, g, count, seed & (2**64 - 1), switches_per_arc, hs,
                                  acc.ctypes.data_as(_P)))
    return [hs[i] for i in range(count)], acc[:count]


def mk_significance(ctx: int, d_hist: int, ng: int, num_classes: int, d_out: int,
                    stream: int = 0) -> None:
    _check(library().mk_significance(ctx, d_hist, ng, num_classes, d_out, stream or None))


def mk_graph_free(g: int) -> None:
    library().mk_graph_free(g)


# -------------------------------------------------------------------- table

def mk_table_build(ctx: int, k: int) -> int:
    h = _P()
    _check(library().mk_table_build(ctx, k, ctypes.byref(h)))
    return h.value


def mk_table_release(ctx: int, k: int) -> None:
    _check(library().mk_table_release(ctx, k))


def mk_table_info(t: int) -> Tuple[int, int, int, float]:
    k, nc, ne, ms = _I32(), _U32(), _U64(), ctypes.c_double()
    _check(library().mk_table_info(t, ctypes.byref(k), ctypes.byref(nc), ctypes.byref(ne),
                                   ctypes.byref(ms)))
    return k.value, nc.value, ne.value, ms.value


def mk_table_class_code(t: int, cid: int) -> int:
    c = _U32()
    _check(library().mk_table_class_code(t, cid, ctypes.byref(c)))
    return c.value


def mk_table_class_codes(t: int) -> np.ndarray:
    nc = mk_table_info(t)[1]
    out = np.empty(nc, dtype=np.uint32)
    _check(library().mk_table_class_codes(t, out.ctypes.data_as(_P), nc))
    return out


def mk_table_lookup(t: int, code: int) -> int:
    c = _U32()
    _check(library().mk_table_lookup(t, code, ctypes.byref(c)))
    return c.value


def mk_table_read(t: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint32)
    _check(library().mk_table_read(t, first, count, out.ctypes.data_as(_P) if count else None))
    return out


def mk_table_core_mult(t: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint8)
    _check(library().mk_table_core_mult(t, first, count,
                                        out.ctypes.data_as(_P) if count else None))
    return out


# -------------------------------------------------------------------- count

def mk_count(ctx: int, g: int, t: int) -> Tuple[np.ndarray, int]:
    nc = mk_table_info(t)[1]
    hist = np.zeros(nc, dtype=np.uint64)
    total = _U64()
    _check(library().mk_count(ctx, g, t, hist.ctypes.data_as(_P), ctypes.byref(total)))
    return hist, total.value


def mk_count_static(ctx: int, g: int, t: int, d_hist: int, stream: int = 0) -> None:
    """H_k of one graph into the device array d_hist (num_classes uint64)
    with no allocation (the library's static device scratch).  Blocks."""
    _check(library().mk_count_static(ctx, g, t, d_hist or None, stream or None))


def mk_static_scratch_bytes() -> int:
    return int(library().mk_static_scratch_bytes())


def _handles(gs: Sequence[int]):
    arr = (_P * max(len(gs), 1))(*gs)
    return arr


def mk_count_batch(ctx: int, gs: Sequence[int], t: int) -> Tuple[np.ndarray, np.ndarray]:
    nc = mk_table_info(t)[1]
    hist = np.zeros((len(gs), nc), dtype=np.uint64)
    totals = np.zeros(len(gs), dtype=np.uint64)
    _check(library().mk_count_batch(ctx, _handles(gs), len(gs), t,
                                    hist.ctypes.data_as(_P) if hist.size else None,
                                    totals.ctypes.data_as(_P) if totals.size else None))
    return hist, totals


def mk_count7(ctx: int, gs: Sequence[int], cap: int = 1 << 16):
    """H_7 of each graph as (codes, counts) arrays sorted by canonical code,
    plus the per-graph totals and the counting kernel's milliseconds."""
    ng = len(gs)
    codes = np.zeros((ng, cap), dtype=np.uint64)
    counts = np.zeros((ng, cap), dtype=np.uint64)
    ncls = np.zeros(ng, dtype=np.int64)
    totals = np.zeros(ng, dtype=np.uint64)
    ms = ctypes.c_double()
    _check(library().mk_count7(ctx, _handles(gs), ng, cap,
                               codes.ctypes.data_as(_P) if codes.size else None,
                               counts.ctypes.data_as(_P) if counts.size else None,
                               ncls.ctypes.data_as(_P) if ng else None,
                               totals.ctypes.data_as(_P) if ng else None, ctypes.byref(ms)))
    out = [(codes[g, :ncls[g]].copy(), counts[g, :ncls[g]].copy()) for g in range(ng)]
    return out, totals, ms.value


def mk_k7_cache_info(ctx: int) -> Tuple[int, int]:
    """(slots, used) of the context's k = 7 canonical-code cache."""
    a, b = _U64(), _U64()
    _check(library().mk_k7_cache_info(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def mk_k7_cache_clear(ctx: int) -> None:
    _check(library().mk_k7_cache_clear(ctx))


def mk_batch_create(ctx: int, gs: Sequence[int], t: int, split_threshold: int = 0,
                    waves_per_cu: int = 0, use_graph: int = 0, units_per_grab: int = 0,
                    units_per_wave: int = 0, method: int = 0, adjacency: int = 0,
                    marks: int = 0) -> int:
    opts = BatchOpts(split_threshold, waves_per_cu, use_graph, units_per_grab, units_per_wave,
                     method, adjacency, marks)
    h = _P()
    _check(library().mk_batch_create(ctx, _handles(gs), len(gs), t, ctypes.byref(opts),
                                     ctypes.byref(h)))
    return h.value


def mk_batch_debug(b: int, flags: int) -> None:
    """Test hook (include/motifs_testing.h): alternative internal paths."""
    _check(library().mk_batch_debug(b, flags))


def mk_batch_run(b: int, d_hist: int = 0, stream: int = 0) -> None:
    """Enqueue one pass.  d_hist: device address (e.g. tensor.data_ptr()) or 0;
    stream: hipStream_t address (e.g. torch stream's cuda_stream) or 0."""
    _check(library().mk_batch_run(b, d_hist or None, stream or None))


def mk_batch_read(b: int, ng: int, num_classes: int) -> Tuple[np.ndarray, np.ndarray]:
    hist = np.zeros((ng, num_classes), dtype=np.uint64)
    totals = np.zeros(ng, dtype=np.uint64)
    _check(library().mk_batch_read(b, hist.ctypes.data_as(_P) if hist.size else None,
                                   totals.ctypes.data_as(_P) if totals.size else None))
    return hist, totals


def mk_batch_stats_get(b: int) -> dict:
    s = BatchStats()
    _check(library().mk_batch_stats_get(b, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in BatchStats._fields_}


def mk_batch_timing(b: int) -> Tuple[float, float]:
    """(whole pass ms, enumeration kernel ms) of the batch's last run."""
    a, e = ctypes.c_double(), ctypes.c_double()
    _check(library().mk_batch_timing(b, ctypes.byref(a), ctypes.byref(e)))
    return a.value, e.value


def mk_batch_free(b: int) -> None:
    library().mk_batch_free(b)


def mk_autotune(ctx: int, gs: Sequence[int], t: int, trials: int = 2) -> Tuple[dict, float, float]:
    """(fastest batch options, its whole-pass ms, the defaults' whole-pass
    ms) for these graphs."""
    o = BatchOpts()
    ms, dms = ctypes.c_double(), ctypes.c_double()
    _check(library().mk_autotune(ctx, _handles(gs), len(gs), t, trials, ctypes.byref(o),
                                 ctypes.byref(ms), ctypes.byref(dms)))
    return {f: getattr(o, f) for f, _ in BatchOpts._fields_}, ms.value, dms.value


# ------------------------------------------------------------------- server

def mk_server_start(ctx: int, hbm_budget_bytes: int = 0, max_slots: int = 0,
                    tick_units: int = 0) -> int:
    opts = ServerOpts(hbm_budget_bytes, max_slots, tick_units)
    h = _P()
    _check(library().mk_server_start(ctx, ctypes.byref(opts), ctypes.byref(h)))
    return h.value


def mk_submit(s: int, g: int, k: int) -> int:
    t = _U64()
    _check(library().mk_submit(s, g, k, ctypes.byref(t)))
    return t.value


def mk_wait(s: int, ticket: int, num_classes: int, timeout_ms: int = -1):
    """(hist, times) of a finished request; raises MotifsError(MK_ETIMEDOUT)."""
    hist = np.zeros(num_classes, dtype=np.uint64)
    times = RequestTimes()
    _check(library().mk_wait(s, ticket, hist.ctypes.data_as(_P), num_classes, timeout_ms,
                             ctypes.byref(times)))
    return hist, {"submit_us": times.submit_us, "admit_us": times.admit_us,
                  "done_us": times.done_us}


def mk_server_stop(s: int) -> None:
    _check(library().mk_server_stop(s))


# ------------------------------------------------------------ handle classes

class Graph:
    def __init__(self, ctx: "Context", row_ptr, col, handle: int = 0):
        self.ctx = ctx
        self.handle = handle or mk_graph_load_csr(ctx.handle, row_ptr, col)
        self.n, self.m, self.max_degree = mk_graph_info(self.handle)

    def read(self) -> Tuple[np.ndarray, np.ndarray]:
        """(row_ptr, col) copied back from the device."""
        return mk_graph_read(self.handle)

    def footprint(self, k: int) -> int:
        return mk_graph_footprint(self.handle, k)

    def free(self) -> None:
        if self.handle:
            mk_graph_free(self.handle)
            self.handle = 0


class Table:
    def __init__(self, ctx: "Context", k: int):
        self.ctx = ctx
        self.handle = mk_table_build(ctx.handle, k)
        self.k, self.num_classes, self.entries, self.build_ms = mk_table_info(self.handle)

    def class_codes(self) -> np.ndarray:
        return mk_table_class_codes(self.handle)

    def class_code(self, cid: int) -> int:
        return mk_table_class_code(self.handle, cid)

    def lookup(self, code: int) -> int:
        return mk_table_lookup(self.handle, code)

    def read(self, first: int, count: int) -> np.ndarray:
        return mk_table_read(self.handle, first, count)

    def core_mult(self, first: int = 0, count: int = -1) -> np.ndarray:
        if count < 0:
            count = self.num_classes - first
        return mk_table_core_mult(self.handle, first, count)


class Batch:
    def __init__(self, ctx: "Context", graphs: Sequence[Graph], table: Table, **opts):
        self.ctx = ctx
        self.graphs = list(graphs)
        self.table = table
        debug = opts.pop("debug_flags", 0)
        self.handle = mk_batch_create(ctx.handle, [g.handle for g in graphs], table.handle,
                                      **opts)
        if debug:
            try:
                mk_batch_debug(self.handle, debug)
            except MotifsError:
                self.free()
                raise

    def run(self, d_hist=None, stream=None) -> None:
        ptr = 0
        if d_hist is not None:
            ptr = d_hist.data_ptr() if hasattr(d_hist, "data_ptr") else int(d_hist)
        sp = 0
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        mk_batch_run(self.handle, ptr, sp)

    def read(self) -> Tuple[np.ndarray, np.ndarray]:
        return mk_batch_read(self.handle, len(self.graphs), self.table.num_classes)

    def stats(self) -> dict:
        return mk_batch_stats_get(self.handle)

    def timing(self) -> Tuple[float, float]:
        return mk_batch_timing(self.handle)

    def free(self) -> None:
        if self.handle:
            mk_batch_free(self.handle)
            self.handle = 0


class Server:
    def __init__(self, ctx: "Context", **opts):
        self.ctx = ctx
        self.handle = mk_server_start(ctx.handle, **opts)

    def submit(self, graph: Graph, k: int) -> int:
        return mk_submit(self.handle, graph.handle, k)

    def wait(self, ticket: int, k: int, timeout_ms: int = -1):
        return mk_wait(self.handle, ticket, NUM_CLASSES[k], timeout_ms)

    def stop(self) -> None:
        if self.handle:
            mk_server_stop(self.handle)
            self.handle = 0


class Context:
    """One device context; tables are cached per k."""

    def __init__(self, device: int = 0):
        self.handle = mk_init(device)
        self.compute_units, self.hbm_bytes = mk_device_info(self.handle)
        self._tables = {}

    def load_graph(self, row_ptr, col) -> Graph:
        return Graph(self, row_ptr, col)

    def table(self, k: int) -> Table:
        if k not in self._tables:
            self._tables[k] = Table(self, k)
        return self._tables[k]

    def release_table(self, k: int) -> None:
        self._tables.pop(k, None)
        mk_table_release(self.handle, k)

    def count(self, graph: Graph, table: Table) -> Tuple[np.ndarray, int]:
        return mk_count(self.handle, graph.handle, table.handle)

    def count_batch(self, graphs: Sequence[Graph], table: Table):
        return mk_count_batch(self.handle, [g.handle for g in graphs], table.handle)

    def count_static(self, graph: Graph, table: Table, d_hist, stream=None) -> None:
        """H_k of one graph into d_hist (a device tensor of num_classes
        int64/uint64, or a device address) without any allocation."""
        ptr = d_hist.data_ptr() if hasattr(d_hist, "data_ptr") else int(d_hist)
        sp = 0
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        mk_count_static(self.handle, graph.handle, table.handle, ptr, sp)

    def count7(self, graphs: Sequence[Graph], cap: int = 1 << 16):
        """H_7: per graph (canonical codes, counts) ascending; totals; kernel ms."""
        return mk_count7(self.handle, [g.handle for g in graphs], cap)

    def k7_cache_info(self) -> Tuple[int, int]:
        return mk_k7_cache_info(self.handle)

    def k7_cache_clear(self) -> None:
        mk_k7_cache_clear(self.handle)

    def batch(self, graphs: Sequence[Graph], table: Table, **opts) -> Batch:
        return Batch(self, graphs, table, **opts)

    def autotune(self, graphs: Sequence[Graph], table: Table, trials: int = 2):
        return mk_autotune(self.handle, [g.handle for g in graphs], table.handle, trials)

    def randomise(self, graph: Graph, count: int, seed: int, switches_per_arc: int = 10):
        """(random graphs, accepted switches): the ensemble of `graph`."""
        hs, acc = mk_randomise(self.handle, graph.handle, count, seed, switches_per_arc)
        return [Graph(self, None, None, handle=h) for h in hs], acc

    def significance(self, d_hist, num_classes: int, d_out, stream=None) -> None:
        """Per class mean / std / z of an ensemble's device histograms
        (ng x num_classes, row 0 the original) into d_out (3 x num_classes
        float64); torch tensors or device addresses."""
        ptr = d_hist.data_ptr() if hasattr(d_hist, "data_ptr") else int(d_hist)
        out = d_out.data_ptr() if hasattr(d_out, "data_ptr") else int(d_out)
        ng = d_hist.shape[0] if hasattr(d_hist, "shape") else None
        if ng is None:
            raise ValueError("d_hist must be a 2-D tensor (ng x num_classes)")
        sp = 0
        if stream is not None:
            sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        mk_significance(self.handle, ptr, ng, num_classes, out, sp)

    def server(self, **opts) -> Server:
        return Server(self, **opts)

    def close(self) -> None:
        if self.handle:
            mk_destroy(self.handle)
            self.handle = 0
            self._tables = {}
