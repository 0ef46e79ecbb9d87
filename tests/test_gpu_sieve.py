"""GPU parity: the HIP sieve (through the C ABI) against the CPU oracle.

Fingerprints are integer (GF(2^64)) results, so the bar is bit-exact equality,
for the whole fingerprint and for the per-iteration values f_L.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2010_08423_amd import inputs
from parity_util import host_threads, oracle_per, say

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


F1 = [(1, 2, 1), (2, 5, 4), (2, 4, 2), (3, 1, 3), (3, 7, 5), (4, 3, 3), (4, 5, 3), (4, 7, 4), (5, 7, 4), (7, 6, 5)]
F2 = [(1, 2, 1), (2, 4, 1), (1, 3, 2), (3, 4, 3), (4, 5, 5)]
F3 = [(1, 2, 1), (2, 3, 2), (3, 6, 5), (2, 5, 1), (1, 4, 2), (4, 5, 3), (5, 6, 5)]
F4 = [(1, 2, 1), (2, 3, 2), (3, 4, 3), (4, 2, 4), (2, 5, 5)]


def arrays(E):
    return (np.array([e[0] for e in E], np.uint32), np.array([e[1] for e in E], np.uint32),
            np.array([e[2] for e in E], np.uint32))


def canonical(src, dst, t):
    keep = src != dst
    trip = np.unique(np.stack([dst[keep], t[keep], src[keep]], axis=1), axis=0)
    return trip[:, 2].astype(np.uint32), trip[:, 0].astype(np.uint32), trip[:, 1].astype(np.uint32)


def check(g_dev, g, k, delta, seed, motif=None, per=False, tuning=None, it_begin=0, it_end=0):
    kw = dict(colour=g.colour, n_colours=g.n_colours, motif=motif) if motif is not None else {}
    if per:
        F, per_o = oracle.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=it_begin, it_end=it_end,
                                per_iteration=True, **kw)
    else:
        F = oracle.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=it_begin, it_end=it_end, **kw)
    r = R.run(g_dev, k, delta, seed, motif=motif, per_iteration=per, tuning=tuning, it_begin=it_begin,
              it_end=it_end)
    assert r.fingerprint == F, (g.name, k, delta, seed, hex(r.fingerprint), hex(F))
    if per:
        assert np.array_equal(r.per_iteration, per_o), (g.name, k, delta, seed)
    return F


def test_symbols_and_version():
    assert b"gfx950" in R.library().rs_version()


def test_graph_upload_canonical():
    rng = np.random.default_rng(0)
    n, m = 50, 4000
    src = rng.integers(0, n, m).astype(np.uint32)
    dst = rng.integers(0, n, m).astype(np.uint32)
    t = rng.integers(1, 20, m).astype(np.uint32)
    g = R.Graph(n, src, dst, t)
    s2, d2, t2 = g.edges()
    cs, cd, ct = canonical(src, dst, t)
    assert np.array_equal(s2, cs) and np.array_equal(d2, cd) and np.array_equal(t2, ct)
    info = g.info()
    assert info["m"] == len(cs)
    assert info["self_loops"] == int((src == dst).sum())
    assert info["duplicates"] == m - info["self_loops"] - len(cs)
    assert info["max_in_degree"] == int(np.bincount(cd, minlength=n).max())


@pytest.mark.parametrize("name,E,n", [("fig1", F1, 8), ("fig2", F2, 6), ("fig3", F3, 7), ("fig4", F4, 6)])
def test_paper_figures(name, E, n):
    s, d, t = arrays(E)
    g = inputs.TemporalGraph(n=n, src=s, dst=d, t=t, name=name)
    gd = R.Graph(n, s, d, t)
    for delta in [0, 1, 2, 3, 10]:
        for k in range(2, n + 1):
            for seed in [1, 77]:
                check(gd, g, k, delta, seed, per=True)


def test_tiny_corpus():
    rr = np.random.default_rng(5)
    for gi in range(60):
        g = inputs.tiny_graph(gi)
        gd = R.Graph.from_inputs(g)
        k = int(rr.integers(2, min(7, g.n) + 1))
        delta = int(rr.integers(0, 5))
        seed = int(rr.integers(0, 2**63))
        motif = inputs.random_motif(k, g.n_colours, rr) if gi % 2 else None
        say("tiny", gi, g.n, g.m, k, delta, motif)
        check(gd, g, k, delta, seed, motif=motif, per=True)


def _medium(seed=11, n=300, m=6000, t_max=50):
    return inputs.uniform_graph(n, m, t_max, seed=seed, name=f"uniform n={n} m={m}")


@pytest.mark.parametrize("E", [8, 16])
@pytest.mark.parametrize("wpb", [1, 4])
@pytest.mark.parametrize("cpl", [1, 2])
def test_tunings(E, wpb, cpl):
    g = _medium()
    gd = R.Graph.from_inputs(g)
    for top in [1, 64, 333]:
        tu = R.Tuning(edges_per_tile=E, top_edges_per_tile=top, chunks_per_launch=cpl, waves_per_block=wpb)
        say("tuning", E, wpb, cpl, top)
        check(gd, g, 7, 3, 1234 + top, tuning=tu, per=(top == 64))


def test_hub_lookback():
    """One vertex with 20,000 in-edges: its segment spans >1000 tiles, so the
    carries travel through long look-back chains."""
    rng = np.random.default_rng(3)
    n = 3000
    m_in = 20000
    src = np.concatenate([rng.integers(1, n, m_in), np.zeros(2000, np.int64), rng.integers(1, n, 4000)])
    dst = np.concatenate([np.zeros(m_in, np.int64), rng.integers(1, n, 2000), rng.integers(1, n, 4000)])
    t = rng.integers(1, 200, src.shape[0])
    g = inputs.TemporalGraph(n=n, src=src.astype(np.uint32), dst=dst.astype(np.uint32), t=t.astype(np.uint32),
                             name="hub")
    gd = R.Graph.from_inputs(g)
    assert gd.info()["max_in_degree"] >= 15000
    for E in (8, 16):
        for delta in (0, 3, 50):
            say("hub", E, delta)
            check(gd, g, 5, delta, 99 + delta, tuning=R.Tuning(edges_per_tile=E), per=True)


def test_iteration_ranges():
    g = _medium(seed=12, n=200, m=3000, t_max=30)
    gd = R.Graph.from_inputs(g)
    k, delta, seed = 8, 4, 4242
    F = check(gd, g, k, delta, seed)
    cuts = [0, 37, 64, 100, 129, 256]
    acc = 0
    for a, b in zip(cuts, cuts[1:]):
        acc ^= check(gd, g, k, delta, seed, it_begin=a, it_end=b, per=True)
    assert acc == F


def test_chunks_per_wave():
    """The last level with one and two chunks per wave. The two-chunk form
    applies only when every chunk group holds an even number of chunks from
    an even chunk; the other cases fall back to one chunk per wave. Both
    forms, over distinct windows (several chunk groups) and over edges (one
    group), path and motif, against the oracle's per-iteration values."""
    g = inputs.add_colours(_medium(seed=13, n=300, m=6000, t_max=40), 4, seed=13)
    gd = R.Graph.from_inputs(g)
    k, delta, seed = 9, 5, 777  # 512 iterations, 8 chunks
    motif = np.array([3, 2, 2, 2], np.uint8)
    cases = [  # chunks per wave, chunks per launch, iteration range
        (2, 8, 0, 0),      # one group of 8: pairs
        (2, 2, 0, 0),      # four groups of 2: pairs over distinct windows
        (2, 4, 128, 384),  # chunks 2..5: pairs
        (2, 3, 0, 0),      # odd groups: one chunk per wave
        (2, 4, 64, 512),   # odd first chunk: one chunk per wave
        (2, 4, 128, 320),  # three chunks: one chunk per wave
        (1, 4, 0, 0),
    ]
    say("chunks per wave: oracle over all iterations")
    ref = {None: oracle_per(g, inputs.Query(k=k, delta=delta, seed=seed), 0, 1 << k, threads=host_threads()),
           "motif": oracle_per(g, inputs.Query(k=k, delta=delta, seed=seed + 1, motif=motif), 0, 1 << k,
                               threads=host_threads())}
    for cpw, cpl, a, b in cases:
        say("chunks per wave", cpw, "per launch", cpl, "range", a, b)
        tu = R.Tuning(chunks_per_wave=cpw, chunks_per_launch=cpl)
        lo, hi = (a, b) if b else (0, 1 << k)
        for key, s_, mot in ((None, seed, None), ("motif", seed + 1, motif)):
            r = R.run(gd, k, delta, s_, motif=mot, tuning=tu, per_iteration=True, it_begin=a, it_end=b)
            want = ref[key][lo:hi]
            assert [int(x) for x in r.per_iteration] == [int(x) for x in want], (cpw, cpl, a, b, key)
            assert r.fingerprint == int(np.bitwise_xor.reduce(want)), (cpw, cpl, a, b, key)


def test_k_extremes():
    g = inputs.tiny_graph(7, n_max=8, m_max=30)
    gd = R.Graph.from_inputs(g)
    for k in (2, 3, 6, 7):
        check(gd, g, k, 2, 5 + k, per=True)
    g2 = inputs.uniform_graph(40, 300, 10, seed=9)
    gd2 = R.Graph.from_inputs(g2)
    for k in (12, 16):
        say("k", k)
        check(gd2, g2, k, 3, 31 + k)


def test_motif_medium():
    g = inputs.add_colours(_medium(seed=13, n=400, m=8000, t_max=40), 4, seed=13)
    gd = R.Graph.from_inputs(g)
    rr = np.random.default_rng(1)
    for k in (4, 6, 9):
        motif = inputs.random_motif(k, 4, rr)
        say("motif", k, motif)
        check(gd, g, k, 5, 500 + k, motif=motif, per=(k < 9))


def test_edge_cases():
    s, d, t = arrays(F1)
    gd = R.Graph(8, s, d, t)
    assert R.run(gd, 9, 2, 1).fingerprint == 0  # k > number of vertices on any path
    e = R.Graph(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert R.run(e, 3, 1, 1).fingerprint == 0
    loops = R.Graph(3, np.array([0, 1], np.uint32), np.array([0, 1], np.uint32), np.array([1, 2], np.uint32))
    assert loops.info()["m"] == 0 and R.run(loops, 2, 1, 1).fingerprint == 0
    r = R.run(gd, 4, 2, 1, it_begin=5, it_end=5)
    assert r.fingerprint == 0
    for bad in [dict(k=1), dict(k=17), dict(k=4, it_begin=3, it_end=2), dict(k=4, it_end=17),
                dict(k=3, motif=[1, 1, 1])]:
        kw = dict(delta=2, seed=1)
        kw.update(bad)
        with pytest.raises(R.RSError):
            R.run(gd, **kw)
    with pytest.raises(R.RSError):
        R.Graph(4, np.array([0], np.uint32), np.array([9], np.uint32), np.array([1], np.uint32))
    with pytest.raises(R.RSError):
        R.Graph(4, np.array([0], np.uint32), np.array([1], np.uint32), np.array([0], np.uint32))
    col = np.array([0, 1, 1, 0, 1, 0, 1, 1], np.uint8)
    gc = R.Graph(8, s, d, t, colour=col, n_colours=2)
    with pytest.raises(R.RSError):
        R.run(gc, 3, 2, 1, motif=[1, 1])  # counts sum to 2, not 3


def test_determinism():
    g = _medium(seed=14)
    gd = R.Graph.from_inputs(g)
    outs = {R.run(gd, 7, 3, 5).fingerprint for _ in range(8)}
    assert len(outs) == 1


def test_config_small_full():
    """Uniform n=1e3, m=1e4, tau=100, delta=5, k=5, seed 1: whole fingerprint
    and every f_L against the oracle."""
    g, q = inputs.config_small()
    gd = R.Graph.from_inputs(g)
    F = check(gd, g, q.k, q.delta, q.seed, per=True)
    assert F != 0
    assert oracle.count_paths(g.n, g.src, g.dst, g.t, q.k, q.delta) > 0


def test_trace_lines(capfd):
    """rs_trace_enable: one stderr line per launch of the plain path, with the
    look-back counters on prefix levels, and the same fingerprint as untraced."""
    g, q = inputs.config_small()
    gd = R.Graph.from_inputs(g)
    F = R.run(gd, q.k, q.delta, q.seed).fingerprint
    capfd.readouterr()
    R.trace_enable(True)
    try:
        Ft = R.run(gd, q.k, q.delta, q.seed).fingerprint
    finally:
        R.trace_enable(False)
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("[rs-trace]")]
    assert Ft == F
    prefix = [ln for ln in lines if " prefix level " in ln]
    # levels 3..k-1 (k >= 4 folds level 2 into level 3's window rows), one chunk group (32 iterations)
    assert len(prefix) == q.k - 3, lines
    assert not any(" prefix level 2 " in ln for ln in prefix)
    assert all("look-back recomputes" in ln for ln in prefix)
    assert sum(" last level " in ln for ln in lines) == 1
    R.run(gd, q.k, q.delta, q.seed)
    assert "[rs-trace]" not in capfd.readouterr().err  # off again


def test_config_path_scale_all_iterations():
    """Chung-Lu n=1e5, m=1e6, delta=10, k=8 at full size in the default launch
    shape (the benchmarked query): all 256 f_L against the oracle, and F =
    XOR of all f_L."""
    g, q = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    r = R.run(gd, q.k, q.delta, q.seed, per_iteration=True)
    assert int(np.bitwise_xor.reduce(r.per_iteration)) == r.fingerprint
    say("cfg2: oracle over all 256 iterations")
    per = oracle_per(g, q, 0, 1 << q.k, threads=host_threads())
    bad = [i for i in range(1 << q.k) if int(r.per_iteration[i]) != int(per[i])]
    assert not bad, bad[:10]
    assert r.fingerprint == int(np.bitwise_xor.reduce(per))


def test_config_motif_scale_sampled():
    """Chung-Lu(2.2) n=1e6, m=1e7, bursty times, 8 colours, motif of k=10
    colours, delta=20, at full size in the default launch shape (four groups
    of four 64-iteration chunks): f_L of 16 iterations, four in each chunk
    group, against the oracle, and F = XOR of all f_L."""
    say("cfg3 graph")
    g, q = inputs.config_motif_scale()
    gd = R.Graph.from_inputs(g)
    say("cfg3 GPU query")
    r = R.run(gd, q.k, q.delta, q.seed, motif=q.motif, per_iteration=True)
    assert int(np.bitwise_xor.reduce(r.per_iteration)) == r.fingerprint
    starts = (62, 317, 517, 1020)  # one range in each group of 256 iterations
    per_call = max(1, host_threads() // len(starts))
    oracle._load()  # build or load once before the calls run side by side
    say("cfg3 oracle iterations", [(a, a + 4) for a in starts], "threads per call", per_call)
    with ThreadPoolExecutor(max_workers=len(starts)) as ex:
        pers = list(ex.map(lambda a: oracle_per(g, q, a, a + 4, threads=per_call), starts))
    say("cfg3 oracle done")
    for a, per in zip(starts, pers):
        assert [int(x) for x in r.per_iteration[a:a + 4]] == [int(x) for x in per], a


def test_graph_create_device_tensors():
    """rs_graph_create_device with torch tensors in HBM (int32 and uint8,
    including duplicates and self-loops): the same canonical graph and the
    same fingerprints as the host upload and the oracle."""
    import torch

    g = inputs.add_colours(inputs.chung_lu_graph(400, 5000, 2.4, 30, seed=77), 5, seed=77)
    rng = np.random.default_rng(78)
    dup = rng.integers(0, g.m, 300)
    src = np.concatenate([g.src, g.src[dup], np.array([3, 9], np.uint32)])
    dst = np.concatenate([g.dst, g.dst[dup], np.array([3, 9], np.uint32)])
    t = np.concatenate([g.t, g.t[dup], np.array([4, 7], np.uint32)])
    gh = R.Graph(g.n, src, dst, t, colour=g.colour, n_colours=g.n_colours)
    dev = torch.device("cuda", 0)
    gt = R.Graph(g.n, torch.from_numpy(src.astype(np.int32)).to(dev), torch.from_numpy(dst.astype(np.int32)).to(dev),
                 torch.from_numpy(t.astype(np.int32)).to(dev), colour=torch.from_numpy(g.colour).to(dev),
                 n_colours=g.n_colours)
    for a, b in zip(gh.edges(), gt.edges()):
        assert np.array_equal(a, b)
    ih, it = gh.info(), gt.info()
    assert ih == it and it["self_loops"] == 2 and it["duplicates"] == 300
    motif = np.array([2, 0, 1, 1, 1], np.uint8)
    for k, delta, mot in ((6, 3, None), (5, 4, motif)):
        F = oracle.sieve(g.n, g.src, g.dst, g.t, k, delta, 91, colour=g.colour, n_colours=g.n_colours, motif=mot)
        assert R.run(gt, k, delta, 91, motif=mot).fingerprint == F
        assert R.run(gh, k, delta, 91, motif=mot).fingerprint == F
