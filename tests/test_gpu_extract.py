"""GPU parity of the extraction of an optimal solution with k fine-grained
queries (Sec. 4.7) and of the constraints it adds to the sieve (removed
vertices, a last timestamp), through the C ABI, against the oracle: the
extracted path (vertices and timestamps) equal to the oracle's, and the
fine-grained outputs under removal / truncation equal, slot for slot, to
the oracle's on the explicitly reduced graph."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2010_08423_amd import inputs
from parity_util import host_threads, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
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


def check_extract(gd, g, k, delta, seed, motif=None, sources=None, targets=None, threads=1):
    want = oracle.extract(g.n, g.src, g.dst, g.t, k, delta, seed, sources=sources, targets=targets, threads=threads,
                          **okw(g, motif))
    verts, times, res = R.extract(gd, k, delta, seed, motif=motif, sources=sources, targets=targets)
    if want is None:
        assert verts is None and not res.yes, (g.name, k)
    else:
        assert res.yes and (verts, times) == (list(want[0]), list(want[1])), (g.name, k, verts, times, want)
    return want


def test_extract_figures():
    for name, claim_k in (("fig_extraction.json", 4), ("fig_fine_grained.json", 4)):
        fx = json.load(open(os.path.join(HERE, "golden", name)))
        E = fx["edges"]
        s, d, t = (np.array([e[i] for e in E], np.uint32) for i in range(3))
        colour = np.array(fx["colour"], np.uint8) if "colour" in fx else None
        g = inputs.TemporalGraph(n=fx["n"], src=s, dst=d, t=t, colour=colour, n_colours=fx.get("n_colours", 0),
                                 name=name)
        gd = R.Graph.from_inputs(g)
        claim = fx["claims"][0]
        for seed in range(3):
            verts, times, res = R.extract(gd, claim_k, fx["delta"], seed,
                                          motif=np.array(claim["motif_count"], np.uint8) if "motif_count" in claim
                                          else None)
            assert verts == claim["path"] and times == [2, 3, 5], (name, verts, times)
        if colour is not None:  # every vertex black: no path agrees
            verts, _, res = R.extract(gd, 4, fx["delta"], 0, motif=np.array([0, 4], np.uint8))
            assert verts is None and not res.yes


def test_extract_tiny_corpus():
    rr = np.random.default_rng(17)
    found = 0
    for gi in range(40):
        g = inputs.tiny_graph(900 + gi, n_colours=3)
        gd = R.Graph.from_inputs(g)
        k = int(rr.integers(2, min(6, g.n) + 1))
        motif = inputs.random_motif(k, g.n_colours, rr) if gi % 2 else None
        delta = int(rr.integers(0, 4))
        if gi % 3 == 0:
            delta = rr.integers(0, 4, g.n).astype(np.uint32)
        sources = sorted(set(rr.integers(0, g.n, 2).tolist())) if gi % 4 == 1 else None
        targets = sorted(set(rr.integers(0, g.n, 3).tolist())) if gi % 5 == 2 else None
        say("extract tiny", gi, k, motif, sources, targets)
        found += check_extract(gd, g, k, delta, int(rr.integers(0, 2**62)), motif=motif, sources=sources,
                               targets=targets) is not None
    assert found >= 10


def test_extract_medium_graphs():
    g = inputs.add_colours(inputs.chung_lu_graph(800, 12000, 2.3, 60, seed=73), 4, seed=73)
    gd = R.Graph.from_inputs(g)
    th = host_threads()
    found = 0
    for k, delta, motif, src, tgt in ((6, 3, None, None, None), (7, 4, np.array([2, 1, 3, 1], np.uint8), None, None),
                                      (5, 2, None, [0, 5, 9], None), (8, 5, None, [1], None),
                                      (6, 3, None, None, [3, 4, 700])):
        say("extract medium", k, delta, motif, src, tgt)
        found += check_extract(gd, g, k, delta, 60 + k, motif=motif, sources=src, targets=tgt, threads=th) is not None
    assert found >= 3


def slot_map(cd, ct, zeta):
    return {(int(cd[e]), int(ct[e])): int(zeta[e]) for e in range(len(cd))}


def test_fine_removed_and_truncated_vs_reduced_graph():
    """rs_run_fine with removed vertices and a last timestamp equals the
    oracle's fine-grained outputs on the graph with those vertices (and their
    edges) and the later edges deleted."""
    g = inputs.add_colours(inputs.chung_lu_graph(500, 6000, 2.3, 40, seed=75), 3, seed=75)
    gd = R.Graph.from_inputs(g)
    cs, cd, ct = oracle.canonical_edges(g.src, g.dst, g.t)
    rr = np.random.default_rng(75)
    for case in range(6):
        k = int(rr.integers(2, 7))
        removed = sorted(set(rr.integers(0, g.n, int(rr.integers(1, 30))).tolist()))
        t_max = int(rr.integers(5, 40)) if case % 2 else 0
        motif = inputs.random_motif(k, g.n_colours, rr) if case % 3 == 1 else None
        delta = int(rr.integers(1, 5))
        rm = np.zeros(g.n, bool)
        rm[removed] = True
        keep = ~rm[cs] & ~rm[cd]
        if t_max:
            keep &= ct <= t_max
        say("fine reduced", case, k, len(removed), t_max, motif)
        zo, ro, Fo = oracle.fine_grained(g.n, cs[keep], cd[keep], ct[keep], k, delta, 80 + case, **okw(g, motif))
        r = R.run_fine(gd, k, delta, 80 + case, motif=motif, removed=removed, t_max=t_max)
        assert r.fingerprint == Fo
        assert np.array_equal(r.reach, ro)
        got = slot_map(cd, ct, r.zeta)
        want = slot_map(*oracle.canonical_edges(cs[keep], cd[keep], ct[keep])[1:], zo)
        assert all(got[s] == want.get(s, 0) for s in got)
        assert all(got[s] == v for s, v in want.items())


def test_extract_rejects_bad_arguments():
    g = inputs.tiny_graph(5)
    gd = R.Graph.from_inputs(g)
    with pytest.raises(Exception):
        R.extract(gd, 1, 2, 0)
    with pytest.raises(Exception):
        R.extract(gd, 3, 2, 0, sources=[g.n + 5])
