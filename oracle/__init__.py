"""Plain CPU oracle for the restless sieve fingerprint (ctypes over oracle.c).

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` import this package. It shares no code
with the GPU library and the GPU library never imports it.

The C source follows arXiv 2010.08423: Eq. (poly-enc:1) (restless-walk
generating function), Eq. (multilinear:1)-(multilinear:3) (sieving with
colour shades), Alg. 1 (sum over subsets L), the exhaustive temporal DFS of
Sec. 5.3 and the determinant closed form of the sieve.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, OpenMP for the
    optional iteration-parallel timing variant)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    u64 = ctypes.c_uint64
    lib.orc_gf_mul.restype = u64
    lib.orc_gf_mul.argtypes = [u64, u64]
    lib.orc_gf_mul_nibble.restype = u64
    lib.orc_gf_mul_nibble.argtypes = [u64, u64]
    lib.orc_gf_pow.restype = u64
    lib.orc_gf_pow.argtypes = [u64, u64]
    lib.orc_gf_inv.restype = u64
    lib.orc_gf_inv.argtypes = [u64]
    lib.orc_mix64.restype = u64
    lib.orc_mix64.argtypes = [u64]
    lib.orc_hash.restype = u64
    lib.orc_hash.argtypes = [u64, u64, _u64p, ctypes.c_int]
    lib.orc_z_table.restype = ctypes.c_int
    lib.orc_z_table.argtypes = [ctypes.c_uint32, _u8p, ctypes.c_uint32, ctypes.c_uint32, _u8p, u64, _u64p]
    graph_args = [ctypes.c_uint32, u64, _u32p, _u32p, _u32p, _u8p, ctypes.c_uint32, ctypes.c_uint32, _u32p, _u8p]
    lib.orc_sieve.restype = ctypes.c_int
    lib.orc_sieve.argtypes = graph_args + [u64, u64, u64, ctypes.c_int, _u64p, _u64p]
    lib.orc_closed_form.restype = ctypes.c_int
    lib.orc_closed_form.argtypes = graph_args + [u64, _u64p, _u64p]
    lib.orc_sieve_ex.restype = ctypes.c_int
    lib.orc_sieve_ex.argtypes = graph_args + [_u8p, _u8p, u64, u64, u64, ctypes.c_int, _u64p, _u64p]
    lib.orc_fine_grained.restype = ctypes.c_int
    lib.orc_fine_grained.argtypes = graph_args + [_u8p, _u8p, u64, u64, u64, ctypes.c_int, _u64p, _u64p, _u32p,
                                                  _u64p]
    lib.orc_fine_literal.restype = ctypes.c_int
    lib.orc_fine_literal.argtypes = graph_args + [u64, u64, u64, ctypes.c_int, _u64p, _u64p, _u32p]
    lib.orc_closed_form_ex.restype = ctypes.c_int
    lib.orc_closed_form_ex.argtypes = graph_args + [_u8p, _u8p, u64, _u64p, _u64p, _u64p, _u64p, _u64p]
    lib.orc_count_paths.restype = ctypes.c_int
    lib.orc_count_paths.argtypes = graph_args + [_u64p]
    lib.orc_gf_det.restype = u64
    lib.orc_gf_det.argtypes = [_u64p, ctypes.c_int]
    lib.orc_gf_det_leibniz.restype = u64
    lib.orc_gf_det_leibniz.argtypes = [_u64p, ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a, typ):
    return a.ctypes.data_as(typ) if a is not None else None


# --- field and hash -------------------------------------------------------

def gf_mul(a: int, b: int) -> int:
    return _load().orc_gf_mul(a, b)


def gf_mul_nibble(a: int, b: int) -> int:
    return _load().orc_gf_mul_nibble(a, b)


def gf_pow(a: int, e: int) -> int:
    return _load().orc_gf_pow(a, e)


def gf_inv(a: int) -> int:
    return _load().orc_gf_inv(a)


def mix64(x: int) -> int:
    return _load().orc_mix64(x)


def keyed_hash(seed: int, tag: int, words) -> int:
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    return _load().orc_hash(seed, tag, _ptr(w, _u64p), len(w))


def gf_det(mat) -> int:
    a = np.ascontiguousarray(np.asarray(mat, dtype=np.uint64))
    return _load().orc_gf_det(_ptr(a, _u64p), a.shape[0])


def gf_det_leibniz(mat) -> int:
    a = np.ascontiguousarray(np.asarray(mat, dtype=np.uint64))
    return _load().orc_gf_det_leibniz(_ptr(a, _u64p), a.shape[0])


# --- graph queries ----------------------------------------------------------

def _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    t = np.ascontiguousarray(t, dtype=np.uint32)
    if not (len(src) == len(dst) == len(t)):
        raise ValueError("src, dst, t must have equal length")
    if np.isscalar(delta):
        delta = np.full(max(n, 1), int(delta), dtype=np.uint32)
    delta = np.ascontiguousarray(delta, dtype=np.uint32)
    col = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
    mot = None if motif is None else np.ascontiguousarray(motif, dtype=np.uint8)
    keep = (src, dst, t, delta, col, mot)
    args = [n, len(src), _ptr(src, _u32p), _ptr(dst, _u32p), _ptr(t, _u32p), _ptr(col, _u8p),
            int(n_colours), int(k), _ptr(delta, _u32p), _ptr(mot, _u8p)]
    return args, keep


def z_table(n, k, seed, colour=None, n_colours=0, motif=None) -> np.ndarray:
    z = np.zeros((max(n, 1), k), dtype=np.uint64)
    col = None if colour is None else np.ascontiguousarray(colour, dtype=np.uint8)
    mot = None if motif is None else np.ascontiguousarray(motif, dtype=np.uint8)
    rc = _load().orc_z_table(n, _ptr(col, _u8p), n_colours, k, _ptr(mot, _u8p), seed, _ptr(z, _u64p))
    if rc:
        raise ValueError(f"orc_z_table rejected the query (rc={rc})")
    return z[:n]


def _mask(n, vertices):
    """uint8 membership array of a vertex list (None: no constraint)."""
    if vertices is None:
        return None
    a = np.zeros(max(n, 1), dtype=np.uint8)
    a[np.asarray(vertices, dtype=np.int64)] = 1
    return a


def sieve(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None,
          it_begin=0, it_end=0, threads=1, per_iteration=False, sources=None, targets=None):
    """Fingerprint F over iterations [it_begin, it_end) (0, 0 = all 2^k).
    sources / targets: vertex lists the paths must start / end in (None: any).
    With per_iteration=True returns (F, array of f_L for the range)."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    F = ctypes.c_uint64(0)
    span = (it_end - it_begin) if (it_begin or it_end) else (1 << k)
    per = np.zeros(max(span, 1), dtype=np.uint64) if per_iteration else None
    sm, tm = _mask(n, sources), _mask(n, targets)
    rc = _load().orc_sieve_ex(*args, _ptr(sm, _u8p), _ptr(tm, _u8p), seed, it_begin, it_end, threads, ctypes.byref(F),
                              _ptr(per, _u64p))
    del keep
    if rc:
        raise ValueError(f"orc_sieve rejected the query (rc={rc})")
    if per_iteration:
        return F.value, per[:span]
    return F.value


UNREACHED = 0xFFFFFFFF


def fine_grained(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None, it_begin=0, it_end=0,
                 threads=1, sources=None, targets=None):
    """Fine-grained oracle (Alg. 1): returns (zeta, reach, F) with zeta[e] the
    zeta_{u,k,i} of the slot (dst, t) of each canonical edge e (order of
    canonical_edges), reach[u] = least i with zeta_{u,k,i} != 0 (UNREACHED if
    none) and F the sum of all zeta."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    m = len(keep[0])
    zeta = np.zeros(max(m, 1), dtype=np.uint64)
    reach = np.zeros(max(n, 1), dtype=np.uint32)
    mc = ctypes.c_uint64(0)
    F = ctypes.c_uint64(0)
    sm, tm = _mask(n, sources), _mask(n, targets)
    rc = _load().orc_fine_grained(*args, _ptr(sm, _u8p), _ptr(tm, _u8p), seed, it_begin, it_end, threads,
                                  _ptr(zeta, _u64p), ctypes.byref(mc), _ptr(reach, _u32p), ctypes.byref(F))
    del keep
    if rc:
        raise ValueError(f"orc_fine_grained rejected the query (rc={rc})")
    return zeta[:mc.value], reach[:n], F.value


def fine_literal(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None, it_begin=0, it_end=0,
                 threads=1):
    """Fine-grained outputs under the literal reading of Eq. (poly-enc:1)
    (y indexed by the predecessor's arrival time): (zeta, reach) as in
    fine_grained, per canonical edge's slot; no aggregate (it cancels)."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    m = len(keep[0])
    zeta = np.zeros(max(m, 1), dtype=np.uint64)
    reach = np.zeros(max(n, 1), dtype=np.uint32)
    mc = ctypes.c_uint64(0)
    rc = _load().orc_fine_literal(*args, seed, it_begin, it_end, threads, _ptr(zeta, _u64p), ctypes.byref(mc),
                                  _ptr(reach, _u32p))
    del keep
    if rc:
        raise ValueError(f"orc_fine_literal rejected the query (rc={rc})")
    return zeta[:mc.value], reach[:n]


def closed_form_slots(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None, sources=None,
                      targets=None):
    """Closed form per slot: (zeta, count, F) with zeta[e] / count[e] the XOR of
    (prod y) det Z_P / the number of (colour-agreeing) restless paths whose
    last edge arrives at the slot (dst, t) of canonical edge e."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    m = len(keep[0])
    zeta = np.zeros(max(m, 1), dtype=np.uint64)
    cnt = np.zeros(max(m, 1), dtype=np.uint64)
    mc = ctypes.c_uint64(0)
    F = ctypes.c_uint64(0)
    npaths = ctypes.c_uint64(0)
    sm, tm = _mask(n, sources), _mask(n, targets)
    rc = _load().orc_closed_form_ex(*args, _ptr(sm, _u8p), _ptr(tm, _u8p), seed, ctypes.byref(F), ctypes.byref(npaths),
                                    _ptr(zeta, _u64p), _ptr(cnt, _u64p), ctypes.byref(mc))
    del keep
    if rc:
        raise ValueError(f"orc_closed_form_ex rejected the query (rc={rc})")
    return zeta[:mc.value], cnt[:mc.value], F.value


def canonical_edges(src, dst, t):
    """The canonical edge list the oracle and the library index by: distinct
    (src, dst, t) triples without self-loops, sorted by (dst, t, src)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    keep = src != dst
    trip = np.unique(np.stack([dst[keep], t[keep], src[keep]], axis=1), axis=0).reshape(-1, 3)
    return trip[:, 2].astype(np.uint32), trip[:, 0].astype(np.uint32), trip[:, 1].astype(np.uint32)


def closed_form(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None):
    """(F, number of restless paths enumerated) from the determinant closed form."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    F = ctypes.c_uint64(0)
    cnt = ctypes.c_uint64(0)
    rc = _load().orc_closed_form(*args, seed, ctypes.byref(F), ctypes.byref(cnt))
    del keep
    if rc:
        raise ValueError(f"orc_closed_form rejected the query (rc={rc})")
    return F.value, cnt.value


def count_paths(n, src, dst, t, k, delta, colour=None, n_colours=0, motif=None) -> int:
    """Number of restless paths with k vertices (agreeing with the motif)."""
    args, keep = _graph_args(n, src, dst, t, colour, n_colours, k, delta, motif)
    cnt = ctypes.c_uint64(0)
    rc = _load().orc_count_paths(*args, ctypes.byref(cnt))
    del keep
    if rc:
        raise ValueError(f"orc_count_paths rejected the query (rc={rc})")
    return cnt.value


# --- fine-grained extraction (Sec. 4.7) --------------------------------------

def extract(n, src, dst, t, k, delta, seed, colour=None, n_colours=0, motif=None, sources=None, targets=None,
            threads=1):
    """Extraction of an optimal solution with k fine-grained queries (Sec. 4.7,
    "using fine-grained oracle"): a restless path with k vertices (agreeing
    with the motif; from a source, to a target when given) whose largest
    timestamp is least. Returns None when the first query finds no path,
    else (vertices, times): vertices u_1..u_k of the path and times[j] the
    timestamp of its edge (u_{j+1} -> u_{j+2}) (0-based j).

    The queries follow the section's generalisation, with the source of the
    reachability instance given directly (walks start only at the sources)
    instead of through an added vertex s':
      * query with k vertices on G: (u_k, i_k) = the slot with least i, then
        least u, among those whose zeta != 0 (optimal: the last edge carries
        the largest timestamp of a restless path);
      * for l = k-1 .. 2: G^l = G without u_{l+1}, .., u_k (and their in- and
        out-edges) and without the edges later than tau^l = i_{l+1}; M^l =
        M^{l+1} minus the colour of u_{l+1}. The query with l vertices on G^l
        gives zeta_{v,l,i}; u_l is the least in-neighbour v of u_{l+1} through
        an edge (v, u_{l+1}, i_{l+1}) that has a slot (v, i) with zeta != 0 in
        its waiting window i_{l+1} - delta(v) <= i <= i_{l+1}, and i_l the
        least such i;
      * u_1 is the least in-neighbour v of u_2 through an edge (v, u_2, i_2)
        that is not removed, is a source, and has the one colour left in M^1.
    Each step's zeta is non-zero only where a path exists, so the pieces join
    into a restless path; a step that finds no candidate met a zero of a
    non-zero polynomial (probability about 2^-57 per slot) and raises."""
    cs, cd, ct = canonical_edges(src, dst, t)
    dv = np.full(max(n, 1), int(delta), dtype=np.int64) if np.isscalar(delta) else np.asarray(delta, dtype=np.int64)
    zeta, reach, _ = fine_grained(n, cs, cd, ct, k, delta, seed, colour, n_colours, motif, threads=threads,
                                  sources=sources, targets=targets)
    ends = range(n) if targets is None else sorted(set(int(x) for x in targets))
    cand = [(int(reach[u]), u) for u in ends if reach[u] != UNREACHED]
    if not cand:
        return None
    i_next, u_next = min(cand)
    verts, times = [u_next], []
    removed = set()
    M = None if motif is None else [int(x) for x in motif]
    src_ok = None if sources is None else set(int(x) for x in sources)
    for l in range(k - 1, 0, -1):
        removed.add(u_next)
        if M is not None:
            M[int(colour[u_next])] -= 1
        # in-edges (v, u_next, i_next) of the last vertex found, in order of v
        into = [int(cs[e]) for e in range(len(cs)) if cd[e] == u_next and ct[e] == i_next]
        into = [v for v in sorted(into) if v not in removed]
        if l == 1:
            ok = [v for v in into if (src_ok is None or v in src_ok) and (M is None or M[int(colour[v])] == 1)]
            if not ok:
                raise RuntimeError("extraction: no start vertex for the last edge")
            verts.append(ok[0])
            times.append(i_next)
            break
        keep = np.array([cs[e] not in removed and cd[e] not in removed and ct[e] <= i_next for e in range(len(cs))],
                        dtype=bool)
        rs, rd, rt = cs[keep], cd[keep], ct[keep]
        zl, _, _ = fine_grained(n, rs, rd, rt, l, delta, seed, colour, n_colours, M, threads=threads, sources=sources)
        slot = {(int(rd[e]), int(rt[e])): int(zl[e]) for e in range(len(rd))}
        pick = None
        for v in into:
            lo = max(1, i_next - int(dv[v]))
            for i in range(lo, i_next + 1):
                if slot.get((v, i), 0):
                    pick = (v, i)
                    break
            if pick:
                break
        if pick is None:
            raise RuntimeError(f"extraction: no predecessor at level {l}")
        times.append(i_next)
        u_next, i_next = pick
        verts.append(u_next)
    return verts[::-1], times[::-1]
