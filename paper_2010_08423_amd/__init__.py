"""Restless-path / restless-motif sieve on MI355X (gfx950).

Thin ctypes binding over ``librestless_sieve.so``; the C ABI is declared in
``include/rs.h``. Every step of a query runs in the library's HIP kernels; this
module only marshals arguments. PyTorch, when present, supplies the current
HIP stream and may hand over device tensors.

Method: Thejaswi, Lauri, Gionis, "Restless reachability problems in temporal
graphs" (arXiv 2010.08423): the restless-walk generating function of
Eq. (poly-enc:1), sieved over subsets L of [k] (Eq. multilinear:1-3, Alg. 1),
in GF(2^64).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librestless_sieve.so")

RS_OK, RS_EINVAL, RS_ENOMEM, RS_EDEVICE, RS_EBUSY, RS_ECANCELED, RS_ENOTFOUND, RS_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
RS_ERETRY = -8
RS_MAX_K = 16

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


class RSError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = f"{what}: {status_str(status)}"
        try:
            extra = _load().rs_last_error().decode()
        except Exception:  # noqa: BLE001
            extra = ""
        if extra:
            msg += f" ({extra})"
        super().__init__(msg)


class _Query(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("delta", ctypes.c_uint32), ("motif_count", _u8p),
                ("seed", ctypes.c_uint64), ("it_begin", ctypes.c_uint64), ("it_end", ctypes.c_uint64)]


class _Result(ctypes.Structure):
    _fields_ = [("fingerprint", ctypes.c_uint64), ("yes", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("device_ms", ctypes.c_float)]


class _Tuning(ctypes.Structure):
    _fields_ = [("edges_per_tile", ctypes.c_uint32), ("top_edges_per_tile", ctypes.c_uint32),
                ("chunks_per_launch", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32),
                ("max_slots", ctypes.c_uint32), ("no_graph", ctypes.c_uint32),
                ("chunks_per_wave", ctypes.c_uint32)]


class _Constraints(ctypes.Structure):
    _fields_ = [("delta_per_vertex", _u32p), ("sources", _u32p), ("n_sources", ctypes.c_uint32),
                ("targets", _u32p), ("n_targets", ctypes.c_uint32), ("removed", _u32p),
                ("n_removed", ctypes.c_uint32), ("t_max", ctypes.c_uint32)]


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("m_input", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("self_loops", ctypes.c_uint64), ("duplicates", ctypes.c_uint64), ("t_min", ctypes.c_uint32),
                ("t_max", ctypes.c_uint32), ("n_colours", ctypes.c_uint32), ("max_in_degree", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("group_edge_updates", ctypes.c_uint64),
                ("streams", ctypes.c_uint32), ("group_max_edges", ctypes.c_uint64)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("deferred", ctypes.c_uint64), ("cancelled", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("inflight", ctypes.c_uint64), ("qps", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("busy_ms", ctypes.c_double),
                ("jobs", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64), ("slices", ctypes.c_uint64)]


# Every symbol include/rs.h declares, with its ctypes signature.
_SIGNATURES = {
    "rs_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "rs_version": (ctypes.c_char_p, []),
    "rs_last_error": (ctypes.c_char_p, []),
    "rs_graph_create": (ctypes.c_int32, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "rs_graph_create_device": (ctypes.c_int32, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_uint32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rs_graph_get_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_GraphInfo)]),
    "rs_graph_edges": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rs_graph_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "rs_query_footprint": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), _u64p]),
    "rs_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_run_ex": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Tuning), _u64p,
                                   ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_run_constrained": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Constraints),
                                            _u64p, ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_run_fine": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Constraints), _u32p,
                                     _u64p, ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_reach_at_most": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Constraints), _u32p,
                                          _u32p, ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_extract": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.POINTER(_Constraints), _u32p,
                                    _u32p, ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_run_literal": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), _u32p, _u32p, _u64p,
                                        ctypes.POINTER(_Result), ctypes.c_void_p]),
    "rs_run_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), _u64p, ctypes.POINTER(_Result),
                                        ctypes.c_void_p]),
    "rs_run_batch": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_Query), ctypes.c_uint32,
                                      ctypes.POINTER(_Result), ctypes.POINTER(_Tuning), ctypes.c_void_p]),
    "rs_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.c_uint32,
                                     ctypes.POINTER(_Tuning)]),
    "rs_autotune_batch": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_Query), ctypes.c_uint32,
                                           ctypes.POINTER(_Tuning)]),
    "rs_profile_enable": (ctypes.c_int32, [ctypes.c_int]),
    "rs_trace_enable": (ctypes.c_int32, [ctypes.c_int]),
    "rs_profile_reset": (ctypes.c_int32, []),
    "rs_lookback_count": (ctypes.c_int32, [ctypes.c_int]),
    "rs_lookback_get": (ctypes.c_int32, [_u64p, _u64p]),
    "rs_profile_get": (ctypes.c_int32, [ctypes.c_char_p, _u64p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "rs_probe_rows": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]),
    "rs_server_create": (ctypes.c_int32, [ctypes.c_uint64, ctypes.POINTER(_ServerOpts),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "rs_server_add_graph": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, _u32p]),
    "rs_server_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(_Query), _u64p]),
    "rs_server_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(_Result), ctypes.c_int32]),
    "rs_server_cancel": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "rs_server_stats_get": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(_ServerStats)]),
    "rs_server_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
}

_lib = None


def _load():
    """Load the HIP library; raises if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue  # reported by missing_symbols(); calling it raises AttributeError
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def library():
    return _load()


def missing_symbols():
    """Names declared by include/rs.h that the built library does not export."""
    lib = _load()
    return [n for n in _SIGNATURES if getattr(lib, n, None) is None]


def status_str(s: int) -> str:
    return _load().rs_status_str(s).decode()


def _check(s, what):
    if s != RS_OK:
        raise RSError(s, what)


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # noqa: BLE001
        pass
    return ctypes.c_void_p(0)


def _is_device_tensor(x):
    return hasattr(x, "is_cuda") and x.is_cuda


@dataclasses.dataclass
class Result:
    fingerprint: int
    yes: bool
    status: int
    device_ms: float
    per_iteration: np.ndarray | None = None


@dataclasses.dataclass
class Tuning:
    edges_per_tile: int = 0
    top_edges_per_tile: int = 0
    chunks_per_launch: int = 0
    waves_per_block: int = 0
    max_slots: int = 0
    no_graph: int = 0
    chunks_per_wave: int = 0

    def _c(self):
        return _Tuning(self.edges_per_tile, self.top_edges_per_tile, self.chunks_per_launch, self.waves_per_block,
                       self.max_slots, self.no_graph, self.chunks_per_wave)


class Graph:
    """A temporal graph resident on the GPU (rs_graph_create / _device)."""

    def __init__(self, n, src, dst, t, colour=None, n_colours=0, stream=None):
        lib = _load()
        h = ctypes.c_void_p()
        st = _stream_handle(stream)
        if _is_device_tensor(src):
            import torch

            src = src.to(torch.int32).contiguous()
            dst = dst.to(torch.int32).contiguous()
            t = t.to(torch.int32).contiguous()
            col = None
            if colour is not None:
                col = colour.to(torch.uint8).contiguous()
            self._keep = (src, dst, t, col)
            s = lib.rs_graph_create_device(int(n), int(src.numel()), src.data_ptr(), dst.data_ptr(), t.data_ptr(),
                                           col.data_ptr() if col is not None else None, int(n_colours), st,
                                           ctypes.byref(h))
        else:
            src = np.ascontiguousarray(src, dtype=np.uint32)
            dst = np.ascontiguousarray(dst, dtype=np.uint32)
            t = np.ascontiguousarray(t, dtype=np.uint32)
            col = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
            s = lib.rs_graph_create(int(n), int(src.shape[0]), src.ctypes.data, dst.ctypes.data, t.ctypes.data,
                                    col.ctypes.data if col is not None else None, int(n_colours), st,
                                    ctypes.byref(h))
        _check(s, "rs_graph_create")
        self._h = h
        self.n = int(n)
        self.n_colours = int(n_colours)

    @classmethod
    def from_inputs(cls, g, stream=None):
        return cls(g.n, g.src, g.dst, g.t, g.colour, g.n_colours, stream=stream)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = _GraphInfo()
        _check(_load().rs_graph_get_info(self._h, ctypes.byref(inf)), "rs_graph_get_info")
        return {f: getattr(inf, f) for f, _ in _GraphInfo._fields_}

    def edges(self):
        m = self.info()["m"]
        s, d, t = (np.zeros(max(m, 1), dtype=np.uint32) for _ in range(3))
        _check(_load().rs_graph_edges(self._h, s.ctypes.data, d.ctypes.data, t.ctypes.data), "rs_graph_edges")
        return s[:m], d[:m], t[:m]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _load().rs_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def _make_query(k, delta, seed, motif=None, it_begin=0, it_end=0):
    mot = None
    if motif is not None:
        mot = np.ascontiguousarray(motif, dtype=np.uint8)
    q = _Query(int(k), int(delta), mot.ctypes.data_as(_u8p) if mot is not None else None, int(seed) & (2**64 - 1),
               int(it_begin), int(it_end))
    return q, mot


def query_struct(query):
    """rs_query for an inputs.Query-like object (k, delta, seed, motif, it_begin, it_end)."""
    return _make_query(query.k, query.delta, query.seed, getattr(query, "motif", None),
                       getattr(query, "it_begin", 0), getattr(query, "it_end", 0))


def footprint(graph: Graph, k, delta, seed=0, motif=None, it_begin=0, it_end=0) -> int:
    q, keep = _make_query(k, delta, seed, motif, it_begin, it_end)
    b = ctypes.c_uint64()
    _check(_load().rs_query_footprint(graph.handle, ctypes.byref(q), ctypes.byref(b)), "rs_query_footprint")
    del keep
    return b.value


def _constraints(delta, sources, targets, removed=None, t_max=0):
    """rs_constraints for a per-vertex delta array, source / target / removed
    vertex lists and a last timestamp (None when there is nothing to
    constrain), and the arrays it points to."""
    per_vertex = not np.isscalar(delta)
    if not per_vertex and sources is None and targets is None and removed is None and not t_max:
        return None, None
    dv = np.ascontiguousarray(delta, dtype=np.uint32) if per_vertex else None

    def ids(x):
        return None if x is None else np.ascontiguousarray(np.asarray(x).reshape(-1), dtype=np.uint32)

    def ptr(a):
        return a.ctypes.data_as(_u32p) if a is not None and len(a) else None

    sv, tv, rv = ids(sources), ids(targets), ids(removed)
    c = _Constraints(dv.ctypes.data_as(_u32p) if dv is not None else None, ptr(sv), 0 if sv is None else len(sv),
                     ptr(tv), 0 if tv is None else len(tv), ptr(rv), 0 if rv is None else len(rv), int(t_max))
    return c, (dv, sv, tv, rv)


def run(graph: Graph, k, delta, seed, motif=None, it_begin=0, it_end=0, tuning: Tuning | None = None,
        per_iteration=False, stream=None, sources=None, targets=None) -> Result:
    """One query on the plain (level-by-level) path: rs_run_ex, or
    rs_run_constrained when delta is a per-vertex array or sources / targets
    (vertex lists the paths must start / end in) are given."""
    c, ckeep = _constraints(delta, sources, targets)
    q, keep = _make_query(k, 0 if c is not None and not np.isscalar(delta) else delta, seed, motif, it_begin, it_end)
    r = _Result()
    per = None
    span = (it_end - it_begin) if (it_begin or it_end) else (1 << k)
    if per_iteration:
        per = np.zeros(max(span, 1), dtype=np.uint64)
    perp = per.ctypes.data_as(_u64p) if per is not None else None
    if c is not None:
        if tuning is not None:
            raise ValueError("launch knobs are not taken with constraints")
        s = _load().rs_run_constrained(graph.handle, ctypes.byref(q), ctypes.byref(c), perp, ctypes.byref(r),
                                       _stream_handle(stream))
        what = "rs_run_constrained"
    else:
        tu = tuning._c() if tuning is not None else None
        s = _load().rs_run_ex(graph.handle, ctypes.byref(q), ctypes.byref(tu) if tu is not None else None, perp,
                              ctypes.byref(r), _stream_handle(stream))
        what = "rs_run_ex"
    del keep, ckeep
    _check(s, what)
    res = Result(r.fingerprint, bool(r.yes), r.status, r.device_ms)
    if per_iteration:
        res.per_iteration = per[:span]
    return res


@dataclasses.dataclass
class FineResult:
    fingerprint: int
    yes: bool
    device_ms: float
    reach: np.ndarray       # uint32 [n]: least time with a path ending there, UNREACHED if none
    zeta: np.ndarray | None  # uint64 [m]: zeta of each canonical edge's slot (dst, t)


UNREACHED = 0xFFFFFFFF


def run_fine(graph: Graph, k, delta, seed, motif=None, it_begin=0, it_end=0, sources=None, targets=None,
             slots=True, stream=None, removed=None, t_max=0) -> FineResult:
    """rs_run_fine: per-slot zeta_{u,k,i} (Alg. 1), reach times and F.
    removed / t_max: vertices no path passes through and the last timestamp
    of the edges used (0 = all)."""
    info = graph.info()
    c, ckeep = _constraints(delta, sources, targets, removed, t_max)
    q, keep = _make_query(k, 0 if not np.isscalar(delta) else delta, seed, motif, it_begin, it_end)
    reach = np.zeros(max(graph.n, 1), dtype=np.uint32)
    zeta = np.zeros(max(info["m"], 1), dtype=np.uint64) if slots else None
    r = _Result()
    s = _load().rs_run_fine(graph.handle, ctypes.byref(q), ctypes.byref(c) if c is not None else None,
                            reach.ctypes.data_as(_u32p), zeta.ctypes.data_as(_u64p) if zeta is not None else None,
                            ctypes.byref(r), _stream_handle(stream))
    del keep, ckeep
    _check(s, "rs_run_fine")
    return FineResult(r.fingerprint, bool(r.yes), r.device_ms, reach[:graph.n],
                      zeta[:info["m"]] if zeta is not None else None)


def run_literal(graph: Graph, k, delta, seed, motif=None, it_begin=0, it_end=0, slots=True,
                stream=None) -> FineResult:
    """rs_run_literal: per-slot zeta_{u,k,i} under the literal reading of Eq.
    (poly-enc:1) (y keyed by the predecessor's arrival time), reach times and
    the XOR of the slot values."""
    info = graph.info()
    dv = None if np.isscalar(delta) else np.ascontiguousarray(delta, dtype=np.uint32)
    q, keep = _make_query(k, delta if dv is None else 0, seed, motif, it_begin, it_end)
    reach = np.zeros(max(graph.n, 1), dtype=np.uint32)
    zeta = np.zeros(max(info["m"], 1), dtype=np.uint64) if slots else None
    r = _Result()
    s = _load().rs_run_literal(graph.handle, ctypes.byref(q), dv.ctypes.data_as(_u32p) if dv is not None else None,
                               reach.ctypes.data_as(_u32p), zeta.ctypes.data_as(_u64p) if zeta is not None else None,
                               ctypes.byref(r), _stream_handle(stream))
    del keep
    _check(s, "rs_run_literal")
    return FineResult(r.fingerprint, bool(r.yes), r.device_ms, reach[:graph.n],
                      zeta[:info["m"]] if zeta is not None else None)


def extract(graph: Graph, k, delta, seed, motif=None, sources=None, targets=None, stream=None):
    """rs_extract: an optimal restless path with k vertices from k
    fine-grained queries (Sec. 4.7). Returns (vertices, times, Result) with
    vertices u_1..u_k and times[j] the timestamp of edge u_{j+1} -> u_{j+2},
    or (None, None, Result) when there is no path."""
    c, ckeep = _constraints(delta, sources, targets)
    q, keep = _make_query(k, 0 if not np.isscalar(delta) else delta, seed, motif)
    verts = np.zeros(max(k, 1), dtype=np.uint32)
    times = np.zeros(max(k - 1, 1), dtype=np.uint32)
    r = _Result()
    s = _load().rs_extract(graph.handle, ctypes.byref(q), ctypes.byref(c) if c is not None else None,
                           verts.ctypes.data_as(_u32p), times.ctypes.data_as(_u32p), ctypes.byref(r),
                           _stream_handle(stream))
    del keep, ckeep
    _check(s, "rs_extract")
    res = Result(r.fingerprint, bool(r.yes), r.status, r.device_ms)
    if not r.yes:
        return None, None, res
    return [int(v) for v in verts[:k]], [int(x) for x in times[:k - 1]], res


def reach_at_most(graph: Graph, k, delta, seed, sources=None, targets=None, stream=None):
    """rs_reach_at_most: (reach times, least number of vertices, Result) over
    the sieves of 2..k vertices."""
    c, ckeep = _constraints(delta, sources, targets)
    q, keep = _make_query(k, 0 if not np.isscalar(delta) else delta, seed)
    reach = np.zeros(max(graph.n, 1), dtype=np.uint32)
    length = np.zeros(max(graph.n, 1), dtype=np.uint32)
    r = _Result()
    s = _load().rs_reach_at_most(graph.handle, ctypes.byref(q), ctypes.byref(c) if c is not None else None,
                                 reach.ctypes.data_as(_u32p), length.ctypes.data_as(_u32p), ctypes.byref(r),
                                 _stream_handle(stream))
    del keep, ckeep
    _check(s, "rs_reach_at_most")
    return reach[:graph.n], length[:graph.n], Result(r.fingerprint, bool(r.yes), r.status, r.device_ms)


def run_noalloc(graph: Graph, k, delta, seed, motif=None, it_begin=0, it_end=0, per_iteration=False,
                stream=None) -> Result:
    """rs_run_noalloc: one query whose workspace lives in the library's
    per-GPU scratch array (no device allocation during the call)."""
    q, keep = _make_query(k, delta, seed, motif, it_begin, it_end)
    r = _Result()
    per = None
    span = (it_end - it_begin) if (it_begin or it_end) else (1 << k)
    if per_iteration:
        per = np.zeros(max(span, 1), dtype=np.uint64)
    s = _load().rs_run_noalloc(graph.handle, ctypes.byref(q), per.ctypes.data_as(_u64p) if per is not None else None,
                               ctypes.byref(r), _stream_handle(stream))
    del keep
    _check(s, "rs_run_noalloc")
    res = Result(r.fingerprint, bool(r.yes), r.status, r.device_ms)
    if per_iteration:
        res.per_iteration = per[:span]
    return res


def run_batch(graphs, queries, tuning: Tuning | None = None, stream=None):
    """rs_run_batch: queries[i] on graphs[i], evaluated together in shared level launches.
    Returns (list of Result, overall status)."""
    nq = len(queries)
    handles = (ctypes.c_void_p * max(nq, 1))(*[g.handle.value for g in graphs])
    qs = (_Query * max(nq, 1))()
    keep = []
    for i, q in enumerate(queries):
        qs[i], mk = query_struct(q)
        keep.append(mk)
    rs = (_Result * max(nq, 1))()
    tu = tuning._c() if tuning is not None else None
    s = _load().rs_run_batch(handles, qs, nq, rs, ctypes.byref(tu) if tu is not None else None,
                             _stream_handle(stream))
    del keep
    out = [Result(rs[i].fingerprint, bool(rs[i].yes), rs[i].status, rs[i].device_ms) for i in range(nq)]
    return out, s


def autotune_batch(graph: Graph, sample_queries) -> Tuning:
    """rs_autotune_batch: the batched launch shape only, timed on the sample as one batch."""
    ns = len(sample_queries)
    qs = (_Query * max(ns, 1))()
    keep = []
    for i, q in enumerate(sample_queries):
        qs[i], mk = query_struct(q)
        keep.append(mk)
    out = _Tuning()
    _check(_load().rs_autotune_batch(graph.handle, qs, ns, ctypes.byref(out)), "rs_autotune_batch")
    del keep
    return Tuning(out.edges_per_tile, out.top_edges_per_tile, out.chunks_per_launch, out.waves_per_block,
                  out.max_slots, out.no_graph, out.chunks_per_wave)


def autotune(graph: Graph, sample_queries) -> Tuning:
    ns = len(sample_queries)
    qs = (_Query * max(ns, 1))()
    keep = []
    for i, q in enumerate(sample_queries):
        qs[i], mk = query_struct(q)
        keep.append(mk)
    out = _Tuning()
    _check(_load().rs_autotune(graph.handle, qs, ns, ctypes.byref(out)), "rs_autotune")
    del keep
    return Tuning(out.edges_per_tile, out.top_edges_per_tile, out.chunks_per_launch, out.waves_per_block,
                  out.max_slots, out.no_graph, out.chunks_per_wave)


# --- kernel timing -------------------------------------------------------------

def profile_enable(on=True):
    _check(_load().rs_profile_enable(1 if on else 0), "rs_profile_enable")


def trace_enable(on=True):
    """rs_trace_enable: per-launch trace lines of the plain path on stderr."""
    _check(_load().rs_trace_enable(1 if on else 0), "rs_trace_enable")


def profile_reset():
    _check(_load().rs_profile_reset(), "rs_profile_reset")


def lookback_count(on: bool):
    """rs_lookback_count: start (and zero) or stop counting look-back events."""
    _check(_load().rs_lookback_count(1 if on else 0), "rs_lookback_count")


def lookback_get():
    """rs_lookback_get: (recomputed predecessor runs, probe rounds without a
    record) since counting was turned on."""
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(_load().rs_lookback_get(ctypes.byref(a), ctypes.byref(b)), "rs_lookback_get")
    return a.value, b.value


def probe_rows(rows, out, waves, steps, mode, stream=None):
    """rs_probe_rows: random 512-byte row reads (mode 0), writes (1) or both
    (2) on device tensors rows [n_rows, 64] (n_rows a power of two) and out
    [waves, 64] of 64-bit integers, enqueued on the stream; the caller times
    it. Bytes moved: waves * steps * (16, 16 or 24) * 512."""
    if rows.dim() != 2 or rows.shape[1] != 64 or rows.element_size() != 8 or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous [n_rows, 64] tensor of 64-bit elements")
    if out.numel() < waves * 64 or out.element_size() != 8 or not out.is_contiguous():
        raise ValueError("out must hold waves x 64 contiguous 64-bit elements")
    _check(_load().rs_probe_rows(rows.data_ptr(), int(rows.shape[0]), out.data_ptr(), int(waves), int(steps),
                                 int(mode), _stream_handle(stream)), "rs_probe_rows")


def profile_get(kernel_class: str):
    """(launches, total_ms, algorithmic_bytes) of a kernel class."""
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    b = ctypes.c_double()
    _check(_load().rs_profile_get(kernel_class.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)),
           "rs_profile_get")
    return n.value, ms.value, b.value


# --- server ------------------------------------------------------------------------

class Server:
    """rs_server_*: continuous batching over resident graphs (0 = the
    library's default for every option)."""

    def __init__(self, hbm_budget, max_inflight=0, group_edge_updates=0, streams=0, group_max_edges=0):
        h = ctypes.c_void_p()
        opts = _ServerOpts(int(max_inflight), int(group_edge_updates), int(streams), int(group_max_edges))
        _check(_load().rs_server_create(int(hbm_budget), ctypes.byref(opts), ctypes.byref(h)), "rs_server_create")
        self._h = h
        self._graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_uint32()
        _check(_load().rs_server_add_graph(self._h, g.handle, ctypes.byref(gid)), "rs_server_add_graph")
        self._graphs.append(g)
        return gid.value

    def submit(self, graph_id, query) -> int:
        q, keep = query_struct(query)
        tk = ctypes.c_uint64()
        s = _load().rs_server_submit(self._h, int(graph_id), ctypes.byref(q), ctypes.byref(tk))
        del keep
        _check(s, "rs_server_submit")
        return tk.value

    def poll(self, ticket, wait_ms=0):
        """Result, or None while pending."""
        r = _Result()
        s = _load().rs_server_poll(self._h, int(ticket), ctypes.byref(r), int(wait_ms))
        if s == RS_ETIMEOUT:
            return None
        _check(s, "rs_server_poll")
        return Result(r.fingerprint, bool(r.yes), r.status, r.device_ms)

    def cancel(self, ticket):
        return _load().rs_server_cancel(self._h, int(ticket))

    def stats(self) -> dict:
        st = _ServerStats()
        _check(_load().rs_server_stats_get(self._h, ctypes.byref(st)), "rs_server_stats_get")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _load().rs_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
