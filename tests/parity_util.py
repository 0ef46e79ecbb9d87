"""Helpers shared by the GPU parity tests: oracle calls spread over the host's
cores (each oracle call is plain single-threaded C unless asked otherwise),
and the per-query oracle fingerprint of an inputs.Query on an inputs graph.

The oracle is the checker here; nothing in this module touches the GPU path.
"""
from __future__ import annotations

import os
import sys
from concurrent.futures import ThreadPoolExecutor

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_threads(cap=16):
    try:
        return max(1, min(cap, len(os.sched_getaffinity(0))))
    except Exception:  # noqa: BLE001
        return max(1, min(cap, os.cpu_count() or 1))


def oracle_kw(g, q):
    return dict(colour=g.colour, n_colours=g.n_colours, motif=q.motif) if q.motif is not None else {}


def oracle_F(g, q, threads=1, delta=None):
    """Oracle fingerprint of query q on graph g over q's iteration range."""
    d = q.delta if delta is None else delta
    return oracle.sieve(g.n, g.src, g.dst, g.t, q.k, d, q.seed, it_begin=q.it_begin, it_end=q.it_end,
                        threads=threads, **oracle_kw(g, q))


def oracle_per(g, q, it_begin, it_end, threads=1):
    """Oracle f_L for the iterations [it_begin, it_end) of query q."""
    return oracle.sieve(g.n, g.src, g.dst, g.t, q.k, q.delta, q.seed, it_begin=it_begin, it_end=it_end,
                        threads=threads, per_iteration=True, **oracle_kw(g, q))[1]


def oracle_many(pairs, workers=None):
    """Oracle fingerprints of many (graph, query) pairs, one single-threaded
    oracle call per pair, run side by side on the host's cores (ctypes drops
    the interpreter lock during each call)."""
    oracle._load()  # build or load once before the calls run side by side
    workers = workers or host_threads()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda gq: oracle_F(gq[0], gq[1]), pairs))


def iterations(q):
    return (q.it_end - q.it_begin) if (q.it_begin or q.it_end) else (1 << q.k)


def oracle_cost(g, q):
    """Edge-updates the oracle performs for q on g (the unit of its run time)."""
    return iterations(q) * max(q.k - 1, 1) * g.m
