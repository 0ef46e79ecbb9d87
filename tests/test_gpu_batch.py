"""GPU: the batched path (rs_run_batch) and the autotuner give the same
fingerprints as the oracle and as the plain path, bit for bit, for every
query alone and in mixes over several graphs, in rounds, in eager and in
hipGraph mode (capture and replays), with explicit, default and autotuned
launch shapes."""
import dataclasses

import numpy as np
import pytest

from paper_2010_08423_amd import inputs
from parity_util import oracle_many, say

pytestmark = pytest.mark.gpu

R = None


def setup_module(module):
    global R
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_08423_amd as lib

    R = lib
    R.library()


def mixed_queries(n_q, n_colours, seed, k_range=(2, 9), delta_range=(0, 6)):
    r = np.random.default_rng(seed)
    out = []
    for i in range(n_q):
        k = int(r.integers(k_range[0], k_range[1] + 1))
        d = int(r.integers(delta_range[0], delta_range[1] + 1))
        motif = inputs.random_motif(k, n_colours, r) if i % 2 else None
        q = inputs.Query(k=k, delta=d, seed=int(r.integers(0, 2**63)), motif=motif)
        if i % 5 == 3:  # a partial iteration range
            total = 1 << k
            a = int(r.integers(0, total))
            b = int(r.integers(a, total + 1))
            q.it_begin, q.it_end = a, b
        out.append(q)
    return out


def plain(gd, q):
    return R.run(gd, q.k, q.delta, q.seed, motif=q.motif, it_begin=q.it_begin, it_end=q.it_end).fingerprint


_GRAPHS = None
_ORACLE = {}


def graphs():
    global _GRAPHS
    if _GRAPHS is None:
        g1 = inputs.add_colours(inputs.uniform_graph(300, 4000, 40, seed=31), 4, seed=31)
        g2 = inputs.add_colours(inputs.chung_lu_graph(500, 9000, 2.3, 60, seed=32), 4, seed=32)
        g3 = inputs.tiny_graph(33, n_max=8, m_max=30, n_colours=4)
        _GRAPHS = [g1, g2, g3]
    return _GRAPHS


def _qkey(q):
    return (q.k, q.delta, q.seed, None if q.motif is None else tuple(int(x) for x in q.motif), q.it_begin, q.it_end)


def oracle_fps(pairs):
    """Oracle fingerprints of (graph, query) pairs, cached across this module's
    tests (graphs come from graphs(), so their identity is stable)."""
    todo = [(g, q) for g, q in pairs if (id(g), _qkey(q)) not in _ORACLE]
    if todo:
        for (g, q), F in zip(todo, oracle_many(todo)):
            _ORACLE[(id(g), _qkey(q))] = (g, F)  # the graph is kept, so its id is not reused
    return [_ORACLE[(id(g), _qkey(q))][1] for g, q in pairs]


def check_batch(gs, gds, qs, which, tuning, label, oracle_every=1):
    """One rs_run_batch of queries qs[i] on graphs gds[which[i]]: every result
    against the plain path alone, and every oracle_every-th result (0: none)
    against the oracle."""
    say(f"[batch] {label}: {len(qs)} queries, tuning={tuning}")
    res, st = R.run_batch([gds[w] for w in which], qs, tuning=tuning)
    say(f"[batch] {label}: status {st}")
    assert st == R.RS_OK
    picked = list(range(0, len(qs), oracle_every)) if oracle_every else []
    want = dict(zip(picked, oracle_fps([(gs[which[i]], qs[i]) for i in picked])))
    for i, (q, w) in enumerate(zip(qs, which)):
        assert res[i].status == R.RS_OK
        assert res[i].fingerprint == plain(gds[w], q), (label, i, q)
        if i in want:
            assert res[i].fingerprint == want[i], (label, i, q)


@pytest.mark.skip(reason="the earlier single-kernel batch design (levels ordered by in-kernel completion "
                  "counters) produced no output for 180 s on this case; the cause was not established and "
                  "that design was removed: batched levels are now ordered by kernel boundaries")
def test_batch_in_kernel_dependency_mix():
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs]
    qs = mixed_queries(24, 4, seed=5)
    check_batch(gs, gds, qs, [i % 3 for i in range(len(qs))], None, "in-kernel-dependency mix", True)


def test_batch_eager_single_query():
    g = graphs()[0]
    gd = R.Graph.from_inputs(g)
    q = inputs.Query(k=5, delta=3, seed=77)
    check_batch([g], [gd], [q], [0], R.Tuning(no_graph=1), "single k=5")


def test_batch_eager_mix():
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs]
    qs = mixed_queries(24, 4, seed=6)
    check_batch(gs, gds, qs, [i % 3 for i in range(len(qs))], R.Tuning(no_graph=1), "eager mix")


@pytest.mark.parametrize("E,wpb,top,slots", [(16, 4, 128, 0), (8, 1, 64, 0), (16, 2, 16, 2), (8, 4, 300, 1),
                                             (16, 4, 1, 3)])
def test_batch_tunings_and_rounds(E, wpb, top, slots):
    """max_slots = 1..3 forces many rounds, so prefix buffers and look-back
    records move between queries and graphs of different sizes."""
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs]
    qs = mixed_queries(12, 4, seed=7 + E + wpb + slots, k_range=(2, 10))
    which = [(i * 7) % 3 for i in range(len(qs))]
    tu = R.Tuning(edges_per_tile=E, waves_per_block=wpb, top_edges_per_tile=top, max_slots=slots, no_graph=1)
    check_batch(gs, gds, qs, which, tu, f"E{E} wpb{wpb} top{top} slots{slots}")


def test_batch_invalid_entries():
    g = graphs()[0]
    gd = R.Graph.from_inputs(g)
    qs = [inputs.Query(k=5, delta=2, seed=1), inputs.Query(k=1, delta=2, seed=1),
          inputs.Query(k=4, delta=1, seed=2, motif=np.array([1, 1, 1, 0], np.uint8)),
          inputs.Query(k=4, delta=1, seed=3, motif=np.array([1, 1, 1, 1], np.uint8))]
    say("[batch] invalid entries")
    res, st = R.run_batch([gd] * 4, qs, tuning=R.Tuning(no_graph=1))
    assert st == R.RS_EINVAL
    assert res[1].status == R.RS_EINVAL and res[2].status == R.RS_EINVAL
    assert res[0].status == R.RS_OK and res[0].fingerprint == plain(gd, qs[0])
    assert res[3].status == R.RS_OK and res[3].fingerprint == plain(gd, qs[3])


def test_batch_empty_and_degenerate():
    """Queries whose F is 0 without any launch: an empty iteration range, and
    a graph whose edges are all self-loops (dropped, so m = 0, and k > n)."""
    g = graphs()[0]
    gd = R.Graph.from_inputs(g)
    loops = inputs.TemporalGraph(n=4, src=np.array([0, 1, 2], np.uint32), dst=np.array([0, 1, 2], np.uint32),
                                 t=np.array([1, 2, 3], np.uint32))
    gl = R.Graph.from_inputs(loops)
    qs = [inputs.Query(k=6, delta=1, seed=1, it_begin=10, it_end=10), inputs.Query(k=5, delta=1, seed=2),
          inputs.Query(k=3, delta=2, seed=3)]
    say("[batch] degenerate entries")
    res, st = R.run_batch([gd, gl, gd], qs, tuning=R.Tuning(no_graph=1))
    assert st == R.RS_OK
    assert res[0].fingerprint == 0 and res[1].fingerprint == 0
    assert res[2].fingerprint == plain(gd, qs[2])


def test_batch_large_k_and_many_chunks():
    g = inputs.uniform_graph(80, 900, 12, seed=41)
    gd = R.Graph.from_inputs(g)
    qs = [inputs.Query(k=12, delta=3, seed=5), inputs.Query(k=10, delta=2, seed=6),
          inputs.Query(k=13, delta=4, seed=7, it_begin=100, it_end=5000)]
    check_batch([g], [gd], qs, [0, 0, 0], R.Tuning(max_slots=40, no_graph=1), "large k")


def test_batch_graph_mode_and_replay():
    """hipGraph mode: first call captures, later calls with the same shape and
    new seeds replay it; each replay is checked against the plain path, with
    eager work and synchronisation in between."""
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs]
    base = mixed_queries(10, 4, seed=11)
    which = [i % 3 for i in range(len(base))]
    for rep in range(4):
        qs = [inputs.Query(k=q.k, delta=q.delta, seed=q.seed + rep, motif=q.motif, it_begin=q.it_begin,
                           it_end=q.it_end) for q in base]
        check_batch(gs, gds, qs, which, None, f"graph replay {rep}")
    # a different shape recaptures
    check_batch(gs, gds, base[:5], which[:5], None, "graph new shape")


def test_autotune_keeps_results():
    g = graphs()[1]
    gd = R.Graph.from_inputs(g)
    qs = mixed_queries(4, 4, seed=13, k_range=(5, 8))
    before = [plain(gd, q) for q in qs]
    assert before == oracle_fps([(g, q) for q in qs])
    say("[batch] autotune")
    tu = R.autotune(gd, qs)
    assert tu.edges_per_tile in (8, 16)
    after = [plain(gd, q) for q in qs]
    assert after == before
    check_batch([g], [gd], qs, [0] * len(qs), None, "after autotune")
    say("[batch] autotune batched shape only")
    tb = R.autotune_batch(gd, qs)
    assert tb.edges_per_tile in (8, 16) and tb.waves_per_block in (1, 2, 4)
    assert [plain(gd, q) for q in qs] == before
    check_batch([g], [gd], qs, [0] * len(qs), None, "after batched autotune")


def test_batch_more_chunk_pairs_than_waves():
    """48 queries of k = 13 (128 chunks each) on one small graph: more
    (query, chunk) pairs in a prefix launch than resident waves, so every
    pair runs on a single wave; results equal the plain path."""
    g = inputs.uniform_graph(60, 700, 10, seed=43)
    gd = R.Graph.from_inputs(g)
    qs = [inputs.Query(k=13, delta=2 + i % 3, seed=500 + i) for i in range(48)]
    check_batch([g], [gd], qs, [0] * len(qs), R.Tuning(no_graph=1), "more pairs than waves", oracle_every=6)


def test_batch_full_size_graph():
    """Four queries of uneven k on the 10^6-edge Chung-Lu graph in one batch
    (every prefix launch partitions the GPU's waves over their chunk pairs),
    bit-identical to the plain path."""
    g, _ = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    qs = [inputs.Query(k=7, delta=10, seed=901), inputs.Query(k=9, delta=25, seed=902),
          inputs.Query(k=5, delta=3, seed=903, motif=np.array([1, 0, 2, 0, 1, 0, 1, 0], np.uint8)),
          inputs.Query(k=8, delta=40, seed=904, it_begin=17, it_end=200)]
    # full ranges of k = 7..9 on 10^6 edges take the oracle hours; the
    # config-4 test checks this graph against the oracle on sampled ranges
    check_batch([g], [gd], qs, [0] * len(qs), R.Tuning(no_graph=1), "full-size graph", oracle_every=0)


def test_batch_config4_mix_vs_oracle():
    """The 64-query mix on the 10^6-edge Chung-Lu graph (k in 4..12, delta in
    2..50, odd queries motif over 8 colours, seeds 100..163), each cut to a
    2-iteration range at a seeded position, in one rs_run_batch with the
    default launch shape through the captured graph (first call captures,
    second replays): every result equals the oracle's."""
    g, _ = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    rr = np.random.default_rng(64)
    qs = []
    for q in inputs.batch_mix():
        a = int(rr.integers(0, (1 << q.k) - 1))
        qs.append(dataclasses.replace(q, it_begin=a, it_end=a + 2))
    say("[batch] config-4 mix: oracle for 64 two-iteration ranges")
    want = oracle_many([(g, q) for q in qs])
    for rep in range(2):
        say(f"[batch] config-4 mix call {rep}")
        res, st = R.run_batch([gd] * len(qs), qs)
        assert st == R.RS_OK
        assert [r.fingerprint for r in res] == want, rep


def test_lookback_counting_keeps_results():
    """With look-back counting on, the batched path (eager and hipGraph) and
    the plain path give the same fingerprints; the counters read back."""
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs[:2]]
    qs = mixed_queries(12, 4, seed=29, k_range=(3, 9))
    which = [gds[i % 2] for i in range(len(qs))]
    want = [plain(gd, q) for gd, q in zip(which, qs)]
    R.lookback_count(True)
    try:
        for no_graph in (1, 0):
            res, st = R.run_batch(which, qs, tuning=R.Tuning(no_graph=no_graph))
            assert st == R.RS_OK and [r.fingerprint for r in res] == want
        assert [plain(gd, q) for gd, q in zip(which, qs)] == want
        rec, rounds = R.lookback_get()
        assert rec >= 0 and rounds >= 0
    finally:
        R.lookback_count(False)
    res, st = R.run_batch(which, qs)
    assert [r.fingerprint for r in res] == want
