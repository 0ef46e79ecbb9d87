"""Pins for the oracle's fine-grained outputs (Alg. 1, FineGrainedOracle,
Sec. 4.5) and its source / destination constraints (the problems of Sec. 3),
against what the paper and the mathematics fix:

* the figure of the fine-grained evaluation scheme (tests/golden): the slots
  at which paths end and the least reach times;
* the closed form per slot: zeta_{u,k,i} equals the XOR over the restless
  paths ending at u at time i of (prod y) det Z_P, bit for bit;
* brute force: the slots with zeta != 0 are exactly the end slots of the
  restless paths a pure-Python enumeration finds (one-sided error: a slot
  that no path ends at is 0 for every seed);
* the sum of zeta over all slots is the aggregated sieve fingerprint;
* the source constraint agrees with the paper's own reductions (the
  k-RestlessReach and k-RestlessMotifReach theorems of Sec. 4.5), whose
  graphs and colourings are built here and run through the motif sieve.
"""
import json
import os
import random

import numpy as np
import pytest

from paper_2010_08423_amd import inputs
from test_oracle_sieve import F1, F2, F3, F4, py_paths, split

HERE = os.path.dirname(os.path.abspath(__file__))
UNREACHED = 0xFFFFFFFF


def end_slots(n, E, k, delta, colour=None, motif=None, sources=None, targets=None):
    """{(u, i)} of the restless paths (brute force) that start in sources and end in targets."""
    out = set()
    for p in py_paths(n, E, k, delta, colour=colour, motif=motif):
        if sources is not None and p[0][0] not in sources:
            continue
        if targets is not None and p[-1][1] not in targets:
            continue
        out.add((p[-1][1], p[-1][2]))
    return out


def nonzero_slots(O, src, dst, t, zeta):
    cs, cd, ct = O.canonical_edges(src, dst, t)
    return {(int(cd[e]), int(ct[e])) for e in range(len(cd)) if zeta[e]}


def test_figure_fine_grained(oracle_mod):
    O = oracle_mod
    fx = json.load(open(os.path.join(HERE, "golden", "fig_fine_grained.json")))
    n, E, delta = fx["n"], fx["edges"], fx["delta"]
    s, d, t = split(E)
    fg = fx["fine_grained"]
    for k_s, slots in fg["nonzero_slots"].items():
        k = int(k_s)
        for seed in range(4):
            zeta, reach, F = O.fine_grained(n, s, d, t, k, delta, seed)
            assert nonzero_slots(O, s, d, t, zeta) == {tuple(x) for x in slots}, (k, seed)
            want = {int(u): i for u, i in fg["reach_time"][k_s].items()}
            got = {u: int(reach[u]) for u in range(n) if reach[u] != UNREACHED}
            assert got == want, (k, seed)
            assert F == O.sieve(n, s, d, t, k, delta, seed)


def _corpus():
    r = random.Random(21)
    for gi in range(120):
        g = inputs.tiny_graph(4000 + gi, n_max=8, m_max=24, t_max=6)
        k = r.randint(2, min(5, g.n))
        if gi % 3 == 2:
            delta = np.array([r.randint(0, 3) for _ in range(g.n)], dtype=np.uint32)
        else:
            delta = r.randint(0, 3)
        motif = inputs.random_motif(k, g.n_colours, np.random.default_rng(gi)) if gi % 2 else None
        sources = sorted(r.sample(range(g.n), r.randint(1, min(2, g.n)))) if gi % 4 in (1, 2) else None
        targets = sorted(r.sample(range(g.n), r.randint(1, min(3, g.n)))) if gi % 5 in (3, 4) else None
        yield gi, g, k, delta, motif, sources, targets, r.getrandbits(63)


def test_fine_grained_equals_closed_form_per_slot(oracle_mod):
    O = oracle_mod
    for gi, g, k, delta, motif, sources, targets, seed in _corpus():
        kw = dict(colour=g.colour, n_colours=g.n_colours, motif=motif, sources=sources, targets=targets)
        zeta, reach, F = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed, **kw)
        cz, cnt, CF = O.closed_form_slots(g.n, g.src, g.dst, g.t, k, delta, seed, **kw)
        assert np.array_equal(zeta, cz), gi
        assert F == CF == O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, **kw), gi


def test_fine_grained_slots_are_the_path_ends(oracle_mod):
    """zeta != 0 exactly at the end slots of the brute-force paths, and R_u is
    the least end time at u; path and motif queries, scalar and per-vertex
    delta, with and without sources and targets."""
    O = oracle_mod
    n_slots = n_empty = 0
    for gi, g, k, delta, motif, sources, targets, seed in _corpus():
        E = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
        want = end_slots(g.n, E, k, delta, colour=g.colour if motif is not None else None, motif=motif,
                         sources=sources, targets=targets)
        kw = dict(colour=g.colour, n_colours=g.n_colours, motif=motif, sources=sources, targets=targets)
        for s_ in (seed, seed + 1):
            zeta, reach, F = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, s_, **kw)
            assert nonzero_slots(O, g.src, g.dst, g.t, zeta) == want, gi
            for u in range(g.n):
                times = [i for (v, i) in want if v == u]
                assert int(reach[u]) == (min(times) if times else UNREACHED), (gi, u)
        n_slots += len(want)
        n_empty += not want
    assert n_slots > 100 and n_empty > 10


def test_fine_grained_range_split(oracle_mod):
    O = oracle_mod
    g = inputs.tiny_graph(77, n_max=8, m_max=28)
    k, delta, seed = 5, 2, 9
    whole, _, F = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed)
    a, _, Fa = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=0, it_end=11)
    b, _, Fb = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=11, it_end=32)
    assert np.array_equal(whole, a ^ b) and F == Fa ^ Fb
    threaded, _, Ft = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed, threads=4)
    assert np.array_equal(threaded, whole) and Ft == F


def _reach_slots(O, n, src, dst, t, zeta, exclude=()):
    return {x for x in nonzero_slots(O, src, dst, t, zeta) if x[0] not in exclude}


def test_source_matches_k_restless_reach_reduction(oracle_mod):
    """Theorem (k-RestlessReach): colour the source s 2 and every other vertex
    1, delete the in-edges of s and ask the motif oracle for M = {1^(k-1), 2}.
    Its non-zero slots are the slots the source-constrained oracle reports."""
    O = oracle_mod
    r = random.Random(31)
    for gi in range(60):
        g = inputs.tiny_graph(5000 + gi, n_max=8, m_max=26, t_max=6)
        k = r.randint(2, min(5, g.n))
        delta = r.randint(0, 3)
        s = r.randrange(g.n)
        colour = np.ones(g.n, dtype=np.uint8)
        colour[s] = 2
        keep = g.dst != s
        motif = np.array([0, k - 1, 1], dtype=np.uint8)
        zr, _, _ = O.fine_grained(g.n, g.src[keep], g.dst[keep], g.t[keep], k, delta, 3 + gi, colour=colour,
                                  n_colours=3, motif=motif)
        zs, _, _ = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, 7 + gi, sources=[s])
        assert _reach_slots(O, g.n, g.src[keep], g.dst[keep], g.t[keep], zr) == \
            _reach_slots(O, g.n, g.src, g.dst, g.t, zs), gi


def test_source_matches_k_restless_motif_reach_reduction(oracle_mod):
    """Theorem (k-RestlessMotifReach): add a vertex s' of a new colour with an
    edge (s', s, i) for every out-edge (s, u, i) of s, and ask the oracle for
    k + 1 vertices and M plus the new colour. Its non-zero slots, other than
    those at s, are the slots of the source-constrained motif oracle."""
    O = oracle_mod
    r = random.Random(32)
    for gi in range(60):
        g = inputs.tiny_graph(6000 + gi, n_max=7, m_max=24, t_max=6)
        k = r.randint(2, min(4, g.n))
        delta = r.randint(0, 3)
        s = r.randrange(g.n)
        motif = inputs.random_motif(k, g.n_colours, np.random.default_rng(gi))
        sp = g.n  # s'
        out_t = sorted({int(tt) for a, b, tt in zip(g.src, g.dst, g.t) if a == s and b != s})
        src2 = np.concatenate([g.src, np.full(len(out_t), sp)]).astype(np.uint32)
        dst2 = np.concatenate([g.dst, np.full(len(out_t), s)]).astype(np.uint32)
        t2 = np.concatenate([g.t, np.array(out_t, dtype=np.int64)]).astype(np.uint32)
        colour2 = np.concatenate([g.colour, [g.n_colours]]).astype(np.uint8)
        motif2 = np.concatenate([motif, [1]]).astype(np.uint8)
        z2, _, _ = O.fine_grained(g.n + 1, src2, dst2, t2, k + 1, delta, 11 + gi, colour=colour2,
                                  n_colours=g.n_colours + 1, motif=motif2)
        zs, _, _ = O.fine_grained(g.n, g.src, g.dst, g.t, k, delta, 13 + gi, colour=g.colour,
                                  n_colours=g.n_colours, motif=motif, sources=[s])
        got = _reach_slots(O, g.n + 1, src2, dst2, t2, z2, exclude=(s,))
        assert got == _reach_slots(O, g.n, g.src, g.dst, g.t, zs, exclude=(s,)), gi


@pytest.mark.parametrize("E,n", [(F1, 8), (F2, 6), (F3, 7), (F4, 6)])
def test_targets_and_sources_split_the_fingerprint(oracle_mod, E, n):
    """F is the XOR over disjoint target sets (and over disjoint source sets)
    of the constrained fingerprints: every path ends (starts) at exactly one
    vertex."""
    O = oracle_mod
    s, d, t = split(E)
    for k in (2, 3, 4):
        for seed in (1, 2):
            F = O.sieve(n, s, d, t, k, 2, seed)
            by_t = 0
            by_s = 0
            for u in range(n):
                by_t ^= O.sieve(n, s, d, t, k, 2, seed, targets=[u])
                by_s ^= O.sieve(n, s, d, t, k, 2, seed, sources=[u])
            assert by_t == F and by_s == F
