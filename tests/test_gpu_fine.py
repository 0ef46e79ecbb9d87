"""GPU parity of the fine-grained outputs (Alg. 1, FineGrainedOracle) and of
the source / destination / per-vertex resting-time constraints (Sec. 2-3,
the reachability reductions of Sec. 4.5 and the at-most-k variant of Sec.
4.6), through the C ABI, against the oracle: per-slot zeta values bit for
bit, reach times exactly, fingerprints bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2010_08423_amd import inputs
from parity_util import host_threads, say

pytestmark = pytest.mark.gpu

R = None
UNREACHED = 0xFFFFFFFF


def setup_module(module):
    global R
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08423_amd as lib

    R = lib
    R.library()


def okw(g, motif):
    return dict(colour=g.colour, n_colours=g.n_colours, motif=motif) if motif is not None else {}


def check_fine(gd, g, k, delta, seed, motif=None, sources=None, targets=None, it_begin=0, it_end=0, threads=1):
    zo, ro, Fo = oracle.fine_grained(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=it_begin, it_end=it_end,
                                     threads=threads, sources=sources, targets=targets, **okw(g, motif))
    r = R.run_fine(gd, k, delta, seed, motif=motif, sources=sources, targets=targets, it_begin=it_begin,
                   it_end=it_end)
    assert r.fingerprint == Fo, (g.name, k, delta)
    assert np.array_equal(r.zeta, zo), (g.name, k, delta)
    assert np.array_equal(r.reach, ro), (g.name, k, delta)
    assert r.yes == bool((ro != UNREACHED).any())
    return r


def test_fine_figures_and_tiny_corpus():
    E = [(1, 2, 1), (2, 4, 1), (1, 3, 2), (3, 4, 3), (4, 5, 5)]
    s, d, t = (np.array([e[i] for e in E], np.uint32) for i in range(3))
    g = inputs.TemporalGraph(n=6, src=s, dst=d, t=t, name="fig fine-grained")
    gd = R.Graph(6, s, d, t)
    for k in (2, 3, 4, 5):
        r = check_fine(gd, g, k, 2, 1 + k)
        if k == 4:
            assert [u for u in range(6) if r.reach[u] != UNREACHED] == [5] and r.reach[5] == 5
    rr = np.random.default_rng(8)
    for gi in range(40):
        g = inputs.tiny_graph(700 + gi, n_colours=3)
        gd = R.Graph.from_inputs(g)
        k = int(rr.integers(2, min(6, g.n) + 1))
        motif = inputs.random_motif(k, g.n_colours, rr) if gi % 2 else None
        delta = int(rr.integers(0, 4))
        if gi % 3 == 0:
            delta = rr.integers(0, 4, g.n).astype(np.uint32)
        sources = sorted(set(rr.integers(0, g.n, 2).tolist())) if gi % 4 == 1 else None
        targets = sorted(set(rr.integers(0, g.n, 2).tolist())) if gi % 5 == 2 else None
        say("fine tiny", gi, k, motif, sources, targets)
        check_fine(gd, g, k, delta, int(rr.integers(0, 2**62)), motif=motif, sources=sources, targets=targets)


def test_fine_medium_graphs():
    g = inputs.add_colours(inputs.chung_lu_graph(800, 12000, 2.3, 60, seed=71), 4, seed=71)
    gd = R.Graph.from_inputs(g)
    for k, delta, motif, src in ((6, 3, None, None), (7, 4, np.array([2, 1, 3, 1], np.uint8), None),
                                 (5, 2, None, [0, 5, 9]), (8, 5, None, [1])):
        say("fine medium", k, delta, motif, src)
        check_fine(gd, g, k, delta, 40 + k, motif=motif, sources=src, threads=host_threads())
    # an iteration range, over a chunk boundary
    check_fine(gd, g, 8, 3, 9, it_begin=50, it_end=140, threads=host_threads())


def test_fine_config_small():
    """Uniform n=1e3, m=1e4, tau=100, delta=5, k=5 (32 iterations): every slot
    and every reach time against the oracle; F equals the plain query's."""
    g, q = inputs.config_small()
    gd = R.Graph.from_inputs(g)
    r = check_fine(gd, g, q.k, q.delta, q.seed, threads=host_threads())
    assert r.fingerprint == R.run(gd, q.k, q.delta, q.seed).fingerprint
    assert (r.reach != UNREACHED).sum() > 0


def test_constrained_plain_runs():
    """rs_run_constrained: sources, targets and per-vertex resting times on the
    plain path, against the oracle's constrained sieve, per iteration."""
    g = inputs.add_colours(inputs.uniform_graph(300, 5000, 40, seed=72), 3, seed=72)
    gd = R.Graph.from_inputs(g)
    rr = np.random.default_rng(73)
    for case in range(10):
        k = int(rr.integers(2, 9))
        dv = rr.integers(0, 8, g.n).astype(np.uint32) if case % 2 else int(rr.integers(0, 8))
        sources = sorted(set(rr.integers(0, g.n, 1 + case).tolist())) if case % 3 != 2 else None
        targets = sorted(set(rr.integers(0, g.n, 5).tolist())) if case % 3 != 1 else None
        motif = inputs.random_motif(k, 3, rr) if case % 4 == 3 else None
        seed = 100 + case
        say("constrained", case, k, sources, targets)
        Fo, per = oracle.sieve(g.n, g.src, g.dst, g.t, k, dv, seed, sources=sources, targets=targets,
                               per_iteration=True, threads=host_threads(), **okw(g, motif))
        r = R.run(gd, k, dv, seed, motif=motif, sources=sources, targets=targets, per_iteration=True)
        assert r.fingerprint == Fo, case
        assert np.array_equal(r.per_iteration, per), case
    # k >= 7 over whole chunk pairs: the last level runs two chunks per wave
    # over the target-restricted list
    dv = rr.integers(0, 8, g.n).astype(np.uint32)
    for case, (k, d, sources, targets, motif) in enumerate((
            (8, dv, [3, 17, 40], list(range(0, g.n, 7)), None),
            (9, 5, None, list(range(1, g.n, 3)), np.array([3, 3, 3], np.uint8)),
            (9, dv, list(range(0, g.n, 11)), None, None))):
        seed = 200 + case
        say("constrained, two chunks per wave", case, k)
        Fo, per = oracle.sieve(g.n, g.src, g.dst, g.t, k, d, seed, sources=sources, targets=targets,
                               per_iteration=True, threads=host_threads(), **okw(g, motif))
        r = R.run(gd, k, d, seed, motif=motif, sources=sources, targets=targets, per_iteration=True)
        assert r.fingerprint == Fo, ("pairs", case)
        assert np.array_equal(r.per_iteration, per), ("pairs", case)


def test_reach_at_most_k():
    """At most k vertices (Sec. 4.6): R_u is the least reach time over the
    sieves of 2..k vertices from the source, and reach_len the least number of
    vertices; each sieve against the oracle's fine-grained output."""
    g = inputs.chung_lu_graph(400, 6000, 2.4, 50, seed=74)
    gd = R.Graph.from_inputs(g)
    s = int(np.bincount(g.src, minlength=g.n).argmax())
    k, delta, seed = 6, 4, 75
    want_r = np.full(g.n, UNREACHED, np.uint64)
    want_len = np.zeros(g.n, np.uint32)
    for kk in range(2, k + 1):
        _, ro, _ = oracle.fine_grained(g.n, g.src, g.dst, g.t, kk, delta, seed, sources=[s],
                                       threads=host_threads())
        hit = (ro != UNREACHED) & (want_len == 0)
        want_len[hit] = kk
        want_r = np.minimum(want_r, ro.astype(np.uint64))
    reach, length, res = R.reach_at_most(gd, k, delta, seed, sources=[s])
    assert np.array_equal(reach.astype(np.uint64), want_r)
    assert np.array_equal(length, want_len)
    assert (length > 0).sum() > 1
