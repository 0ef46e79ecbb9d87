"""GPU parity of the fine-grained sieve under the literal reading of Eq.
(poly-enc:1) (y keyed by the predecessor's arrival time, one product per
window term), through the C ABI, against the oracle: per-slot zeta bit for
bit, reach times exactly, and the XOR of the slot values."""
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


def slot_xor(src, dst, t, zeta):
    """XOR of the values of the distinct slots (each slot once)."""
    cs, cd, ct = oracle.canonical_edges(src, dst, t)
    first = np.ones(len(cd), bool)
    first[1:] = (cd[1:] != cd[:-1]) | (ct[1:] != ct[:-1])
    return int(np.bitwise_xor.reduce(zeta[first])) if len(cd) else 0


def check_literal(gd, g, k, delta, seed, motif=None, it_begin=0, it_end=0, threads=1):
    zo, ro = oracle.fine_literal(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=it_begin, it_end=it_end,
                                 threads=threads, **okw(g, motif))
    r = R.run_literal(gd, k, delta, seed, motif=motif, it_begin=it_begin, it_end=it_end)
    assert np.array_equal(r.zeta, zo), (g.name, k, delta)
    assert np.array_equal(r.reach, ro), (g.name, k, delta)
    assert r.fingerprint == slot_xor(g.src, g.dst, g.t, zo)
    assert r.yes == bool((ro != UNREACHED).any())
    return r


def test_literal_figure_and_cancellation():
    E = [(1, 2, 1), (2, 4, 1), (1, 3, 2), (3, 4, 3), (4, 5, 5)]
    s, d, t = (np.array([e[i] for e in E], np.uint32) for i in range(3))
    g = inputs.TemporalGraph(n=6, src=s, dst=d, t=t, name="fig fine-grained")
    gd = R.Graph(6, s, d, t)
    for k in (2, 3, 4, 5):
        r = check_literal(gd, g, k, 2, 3 + k)
        if k == 4:
            assert [u for u in range(6) if r.reach[u] != UNREACHED] == [5] and r.reach[5] == 5
    # s -> v at 3, v -> u at 4 and 5: both end slots hold the same value
    s, d, t = (np.array(x, np.uint32) for x in ([0, 1, 1], [1, 2, 2], [3, 4, 5]))
    g = inputs.TemporalGraph(n=3, src=s, dst=d, t=t, name="cancellation")
    gd = R.Graph(3, s, d, t)
    for seed in range(4):
        r = check_literal(gd, g, 3, 2, seed)
        assert r.zeta[1] == r.zeta[2] != 0 and r.fingerprint == 0


def test_literal_tiny_corpus():
    rr = np.random.default_rng(31)
    for gi in range(40):
        g = inputs.tiny_graph(1200 + gi, n_colours=3)
        gd = R.Graph.from_inputs(g)
        k = int(rr.integers(2, min(6, g.n) + 1))
        motif = inputs.random_motif(k, g.n_colours, rr) if gi % 2 else None
        delta = rr.integers(0, 4, g.n).astype(np.uint32) if gi % 3 == 0 else int(rr.integers(0, 4))
        say("literal tiny", gi, k, motif)
        check_literal(gd, g, k, delta, int(rr.integers(0, 2**62)), motif=motif)


def test_literal_hub_slots_span_tiles():
    """A vertex receiving 100 edges at one time (its slot spans several
    16-edge tiles) and long windows of a busy source."""
    rr = np.random.default_rng(5)
    src, dst, t = [], [], []
    for v in range(1, 101):
        src.append(v), dst.append(0), t.append(7)  # hub slot (0, 7)
        src.append(0), dst.append(v), t.append(int(rr.integers(1, 12)))
        src.append(v), dst.append(int(rr.integers(101, 140))), t.append(int(rr.integers(5, 15)))
    for _ in range(400):
        a, b = (int(x) for x in rr.integers(0, 140, 2))
        if a != b:
            src.append(a), dst.append(b), t.append(int(rr.integers(1, 15)))
    g = inputs.TemporalGraph(n=140, src=np.array(src, np.uint32), dst=np.array(dst, np.uint32),
                             t=np.array(t, np.uint32), name="hub")
    gd = R.Graph.from_inputs(g)
    for k, delta in ((3, 4), (5, 6), (6, 10), (7, 3)):
        say("literal hub", k, delta)
        check_literal(gd, g, k, delta, 11 * k, threads=host_threads())


def test_literal_medium_graphs():
    g = inputs.add_colours(inputs.chung_lu_graph(800, 12000, 2.3, 60, seed=77), 4, seed=77)
    gd = R.Graph.from_inputs(g)
    th = host_threads()
    for k, delta, motif in ((6, 3, None), (7, 4, np.array([2, 1, 3, 1], np.uint8)), (8, 5, None)):
        say("literal medium", k, delta, motif)
        check_literal(gd, g, k, delta, 90 + k, motif=motif, threads=th)
    check_literal(gd, g, 8, 3, 9, it_begin=50, it_end=140, threads=th)  # over a chunk boundary


def test_literal_path_scale_sampled():
    """The Chung-Lu n=1e5, m=1e6, delta=10, k=8 graph at full size: the two
    iterations on either side of a chunk boundary against the oracle, slot
    for slot."""
    g, q = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    say("literal path-scale iterations 127..128")
    check_literal(gd, g, q.k, q.delta, q.seed, it_begin=127, it_end=129, threads=host_threads())
