"""GPU: the server (rs_server_*) returns, for every query of a stream of
arrivals, the oracle's fingerprint and the fingerprint the plain path gives
for it alone, whether the query runs in a group (shared batched launches) or
alone on one of several concurrent worker streams, while it admits queries
against an HBM budget, cancels, and is driven from several threads."""
import dataclasses
import threading
import time

import numpy as np
import pytest

from paper_2010_08423_amd import inputs
from parity_util import oracle_cost, oracle_many, say

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
        if i % 5 == 3:
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
    """Oracle fingerprints of (graph, query) pairs, cached across the tests of
    this module (the same arrivals recur under several server options)."""
    todo = [(g, q) for g, q in pairs if (id(g), _qkey(q)) not in _ORACLE]
    if todo:
        say(f"[server] oracle for {len(todo)} queries")
        for (g, q), F in zip(todo, oracle_many(todo)):
            _ORACLE[(id(g), _qkey(q))] = (g, F)  # the graph is kept, so its id is not reused
    return [_ORACLE[(id(g), _qkey(q))][1] for g, q in pairs]


@pytest.mark.parametrize("label,opts", [
    ("grouped", dict(group_edge_updates=2_000_000)),
    ("grouped small graphs, g2 alone", dict(group_max_edges=5000, streams=3)),
    ("all alone, 6 streams", dict(group_edge_updates=1, streams=6)),
])
def test_server_alone_vs_mix(label, opts):
    gs = graphs()
    gds = [R.Graph.from_inputs(g) for g in gs]
    qs = mixed_queries(30, 4, seed=17, k_range=(2, 10))
    which = [i % 3 for i in range(len(qs))]
    alone = [plain(gds[w], q) for q, w in zip(qs, which)]
    want = oracle_fps([(gs[w], q) for q, w in zip(qs, which)])
    assert alone == want
    say(f"[server] 30 arrivals over 3 graphs, {label}")
    srv = R.Server(hbm_budget=8 << 30, **opts)
    ids = [srv.add_graph(gd) for gd in gds]
    tickets = []
    for q, w in zip(qs, which):
        tickets.append(srv.submit(ids[w], q))
        time.sleep(0.001)  # arrivals while earlier work is on the device
    got = [srv.poll(t, wait_ms=60000) for t in tickets]
    assert all(r is not None and r.status == R.RS_OK for r in got)
    assert [r.fingerprint for r in got] == want
    st = srv.stats()
    assert st["completed"] == len(qs) and st["jobs"] >= 1
    assert st["p99_ms"] >= st["p50_ms"] > 0
    assert 0 < st["held_bytes"] <= 8 << 30
    srv.close()


def test_server_budget_deferral_cancel_and_threads():
    g = graphs()[1]
    gd = R.Graph.from_inputs(g)
    qs = mixed_queries(16, 4, seed=19, k_range=(6, 9))
    alone = [plain(gd, q) for q in qs]
    assert alone == oracle_fps([(g, q) for q in qs])
    fp = max(R.footprint(gd, q.k, q.delta) for q in qs)
    # four workers, room for about two queries at a time: the rest must wait
    say("[server] budget for about two queries, 4 workers, 4 submitting threads")
    srv = R.Server(hbm_budget=int(fp * 2.2), max_inflight=64, group_edge_updates=1_000_000, streams=4)
    gid = srv.add_graph(gd)
    with pytest.raises(R.RSError):
        srv.submit(gid, inputs.Query(k=17, delta=1, seed=1))  # invalid k
    tickets = [None] * len(qs)

    def sub(lo, hi):
        for i in range(lo, hi):
            tickets[i] = srv.submit(gid, qs[i])

    th = [threading.Thread(target=sub, args=(a, a + 4)) for a in range(0, 16, 4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    extra = srv.submit(gid, qs[0])
    srv.cancel(extra)
    r_extra = srv.poll(extra, wait_ms=60000)
    assert r_extra.status in (R.RS_ECANCELED, R.RS_OK)
    got = [srv.poll(t, wait_ms=120000) for t in tickets]
    assert [r.fingerprint for r in got] == alone
    st = srv.stats()
    assert st["deferred"] > 0 and st["completed"] >= len(qs)
    assert st["held_bytes"] <= int(fp * 2.2)
    small = R.Server(hbm_budget=1024)
    gid2 = small.add_graph(gd)
    with pytest.raises(R.RSError):
        small.submit(gid2, qs[0])  # can never fit
    small.close()
    srv.close()


def test_server_config5_stream_vs_oracle():
    """The served stream of the 4-graph workload (Poisson arrivals, k in
    4..12, delta in 1..100, 30 % motif queries over 8 colours), on its two
    smaller graphs (m = 10^4 uniform, m = 10^5 Chung-Lu 2.5, tau = m/100):
    64 arrivals submitted at their (compressed) arrival times while earlier
    ones run. A query whose oracle run would exceed 10^7 edge-updates keeps a
    2-iteration range of its sieve at a seeded position (the range is part of
    the served query). Every result equals the oracle's and the plain path's
    for the query alone."""
    gs = inputs.served_graphs(sizes=(10_000, 100_000))
    gds = [R.Graph.from_inputs(g) for g in gs]
    stream = inputs.served_stream(200.0, 60.0, len(gs))[:64]
    rr = np.random.default_rng(55)
    arrivals = []
    for ta, gi, q in stream:
        if oracle_cost(gs[gi], q) > 10_000_000:
            a = int(rr.integers(0, (1 << q.k) - 1))
            q = dataclasses.replace(q, it_begin=a, it_end=a + 2)
        arrivals.append((ta, gi, q))
    want = oracle_fps([(gs[gi], q) for _, gi, q in arrivals])
    alone = [plain(gds[gi], q) for _, gi, q in arrivals]
    assert alone == want
    say(f"[server] config-5 stream: {len(arrivals)} arrivals on m = {[g.m for g in gs]}")
    srv = R.Server(hbm_budget=16 << 30)
    ids = [srv.add_graph(gd) for gd in gds]
    tickets = []
    t0 = time.perf_counter()
    for ta, gi, q in arrivals:
        d = t0 + ta / 10.0 - time.perf_counter()  # arrival times compressed tenfold
        if d > 0:
            time.sleep(d)
        tickets.append(srv.submit(ids[gi], q))
    got = [srv.poll(t, wait_ms=120000) for t in tickets]
    assert all(r is not None and r.status == R.RS_OK for r in got)
    assert [r.fingerprint for r in got] == want
    st = srv.stats()
    assert st["completed"] == len(arrivals)
    srv.close()


def test_server_chunk_boundary_slices():
    """Queries whose work exceeds the group cap run as slices of whole
    64-iteration chunks in successive groups (their fingerprints XOR to the
    query's); a small query that arrives while a long one is being sliced
    joins the next group and completes first. Every result equals the
    oracle's and the plain path's."""
    g = graphs()[0]  # m = 4000
    gd = R.Graph.from_inputs(g)
    r = np.random.default_rng(23)
    qs = [inputs.Query(k=int(r.integers(7, 11)), delta=int(r.integers(0, 6)), seed=int(r.integers(0, 2**62)),
                       motif=inputs.random_motif(8, 4, r) if i % 3 == 1 else None) for i in range(10)]
    qs = [dataclasses.replace(q, k=8) if q.motif is not None else q for q in qs]
    big = inputs.Query(k=12, delta=3, seed=5)
    small = inputs.Query(k=4, delta=2, seed=6)
    allq = qs + [big, small]
    want = oracle_fps([(g, q) for q in allq])
    assert [plain(gd, q) for q in allq] == want
    say("[server] slices: 10 queries of k 7..10, then k=12 followed by k=4, cap 1e7 edge-updates")
    srv = R.Server(hbm_budget=8 << 30, group_edge_updates=10_000_000, streams=1)
    gid = srv.add_graph(gd)
    tickets = [srv.submit(gid, q) for q in qs]
    got = [srv.poll(t, wait_ms=60000) for t in tickets]
    assert [x.fingerprint for x in got] == want[:10]
    t_big = srv.submit(gid, big)
    time.sleep(0.002)
    t_small = srv.submit(gid, small)
    r_small = srv.poll(t_small, wait_ms=60000)
    r_big = srv.poll(t_big, wait_ms=60000)
    assert r_big.fingerprint == want[10] and r_small.fingerprint == want[11]
    assert r_small.device_ms < r_big.device_ms  # latencies: the small one finished first
    st = srv.stats()
    assert st["completed"] == 12 and st["slices"] > 12
    srv.close()
