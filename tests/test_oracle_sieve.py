"""Pins for the oracle's sieve against brute force and the closed form.

* An independent Python enumeration of restless paths (straight from the
  definitions of Sec. 2) pins the C DFS.
* The determinant closed form F = XOR_P Y_P det Z_P pins the sieve bit for bit.
* F != 0 exactly when a (colour-agreeing) restless path exists.
* NO instances give F == 0 for every seed (one-sided error).
* Invariances: edge order, duplicates, self-loops, delta saturation, equal
  timestamps, colour-excluded vertices, iteration-range splits.
"""
import itertools
import random

import numpy as np
import pytest

from paper_2010_08423_amd import inputs

F1 = [(1, 2, 1), (2, 5, 4), (2, 4, 2), (3, 1, 3), (3, 7, 5), (4, 3, 3), (4, 5, 3), (4, 7, 4), (5, 7, 4), (7, 6, 5)]
F2 = [(1, 2, 1), (2, 4, 1), (1, 3, 2), (3, 4, 3), (4, 5, 5)]
F3 = [(1, 2, 1), (2, 3, 2), (3, 6, 5), (2, 5, 1), (1, 4, 2), (4, 5, 3), (5, 6, 5)]
F4 = [(1, 2, 1), (2, 3, 2), (3, 4, 3), (4, 2, 4), (2, 5, 5)]


def split(E):
    return ([e[0] for e in E], [e[1] for e in E], [e[2] for e in E])


def py_paths(n, E, k, delta, colour=None, motif=None):
    """All restless paths with k vertices, by brute force over edge sequences."""
    E = sorted(set((a, b, c) for a, b, c in E if a != b))
    d = (lambda v: delta) if np.isscalar(delta) else (lambda v: int(delta[v]))
    out = []
    for seq in itertools.product(E, repeat=k - 1):
        ok = True
        for p in range(k - 2):
            (a, b, t1), (c, e, t2) = seq[p], seq[p + 1]
            if b != c or not (0 <= t2 - t1 <= d(b)):
                ok = False
                break
        if not ok:
            continue
        verts = [seq[0][0]] + [s[1] for s in seq]
        if len(set(verts)) != k:
            continue
        if motif is not None:
            cnt = np.bincount([colour[v] for v in verts], minlength=len(motif))
            if len(cnt) != len(motif) or not np.array_equal(cnt, motif):
                continue
        out.append(tuple(seq))
    return out


@pytest.mark.parametrize("E,n", [(F1, 8), (F2, 6), (F3, 7), (F4, 6)])
@pytest.mark.parametrize("delta", [0, 1, 2, 3])
def test_dfs_matches_python_enumeration(oracle_mod, E, n, delta):
    s, d, t = split(E)
    for k in range(2, min(n, 7) + 1):
        if k > 5 and len(E) > 8:
            continue  # keep the python product small
        assert oracle_mod.count_paths(n, s, d, t, k, delta) == len(py_paths(n, E, k, delta))


def test_dfs_fig1_counts(oracle_mod):
    """Counts on the Sec. 3 example graph, delta = 2: the k = 6 paths are
    exactly the two highlighted in the figure's left and right panels."""
    s, d, t = split(F1)
    assert [oracle_mod.count_paths(8, s, d, t, k, 2) for k in range(2, 8)] == [10, 11, 10, 5, 2, 0]
    six = {tuple([p[0][0]] + [e[1] for e in p]) for p in py_paths(8, F1, 6, 2)}
    assert six == {(1, 2, 4, 5, 7, 6), (1, 2, 4, 3, 7, 6)}


@pytest.mark.parametrize("E,n", [(F1, 8), (F2, 6), (F3, 7), (F4, 6)])
def test_sieve_equals_closed_form_fixtures(oracle_mod, E, n):
    O = oracle_mod
    s, d, t = split(E)
    for delta in [0, 1, 2, 3, 10]:
        for k in range(2, n + 1):
            for seed in [1, 2]:
                F = O.sieve(n, s, d, t, k, delta, seed)
                C, npaths = O.closed_form(n, s, d, t, k, delta, seed)
                assert F == C
                assert (F != 0) == (npaths > 0)


def test_sieve_equals_closed_form_random_corpus(oracle_mod):
    O = oracle_mod
    r = random.Random(77)
    n_yes = n_no = 0
    for gi in range(160):
        g = inputs.tiny_graph(gi)
        k = r.randint(2, min(6, g.n))
        delta = r.randint(0, 4)
        seed = r.getrandbits(64)
        motif = None
        if gi % 2:
            motif = inputs.random_motif(k, g.n_colours, np.random.default_rng(gi))
        kw = dict(colour=g.colour, n_colours=g.n_colours, motif=motif)
        F = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, **kw)
        C, _ = O.closed_form(g.n, g.src, g.dst, g.t, k, delta, seed, **kw)
        cnt = O.count_paths(g.n, g.src, g.dst, g.t, k, delta, **kw)
        assert F == C, (gi, k, delta)
        assert (F != 0) == (cnt > 0), (gi, k, delta)
        n_yes += cnt > 0
        n_no += cnt == 0
    assert n_yes > 20 and n_no > 20


def test_per_vertex_delta(oracle_mod):
    O = oracle_mod
    r = random.Random(8)
    for gi in range(40):
        g = inputs.tiny_graph(500 + gi)
        k = r.randint(2, min(5, g.n))
        delta = np.array([r.randint(0, 3) for _ in range(g.n)], dtype=np.uint32)
        F = O.sieve(g.n, g.src, g.dst, g.t, k, delta, 99)
        C, _ = O.closed_form(g.n, g.src, g.dst, g.t, k, delta, 99)
        E = list(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))
        assert F == C
        assert O.count_paths(g.n, g.src, g.dst, g.t, k, delta) == len(py_paths(g.n, E, k, delta))


NO_INSTANCES = [
    ("fig1 k=7", F1, 8, 7, 2, None, None),
    ("fig2 delta=1", F2, 6, 4, 1, None, None),
    ("fig3 M={b,b,b,b}", F3, 7, 4, 2, [1, 0, 1, 1, 1, 1, 1], [0, 4]),
    ("fig4 k=5 (walks of 4 edges exist)", F4, 6, 5, 2, None, None),
    ("fig4 k=6 (the walk of 5 edges exists)", F4, 6, 6, 2, None, None),
]


@pytest.mark.parametrize("name,E,n,k,delta,colour,motif", NO_INSTANCES)
def test_one_sided_error(oracle_mod, name, E, n, k, delta, colour, motif):
    O = oracle_mod
    s, d, t = split(E)
    kw = {}
    if motif is not None:
        kw = dict(colour=colour, n_colours=len(motif), motif=motif)
    assert O.count_paths(n, s, d, t, k, delta, **kw) == 0
    for seed in range(100):
        assert O.sieve(n, s, d, t, k, delta, seed, **kw) == 0


def test_k2_by_hand(oracle_mod):
    """k = 2: F = XOR over edges e = (v,u,t), v != u, of
    y_{e,1} (z_{v,1} z_{u,2} + z_{v,2} z_{u,1}), independent of delta."""
    O = oracle_mod
    g = inputs.tiny_graph(3, n_max=6, m_max=20)
    seed = 4242
    z = O.z_table(g.n, 2, seed)
    expect = 0
    for v, u, tt in sorted(set(zip(g.src.tolist(), g.dst.tolist(), g.t.tolist()))):
        if v == u:
            continue
        y = O.keyed_hash(seed, ord("Y"), [v | (u << 32), tt | (1 << 32)])
        expect ^= O.gf_mul(y, O.gf_mul(int(z[v, 0]), int(z[u, 1])) ^ O.gf_mul(int(z[v, 1]), int(z[u, 0])))
    for delta in [0, 3, 100]:
        assert O.sieve(g.n, g.src, g.dst, g.t, 2, delta, seed) == expect


def test_z_table_definition(oracle_mod):
    O = oracle_mod
    z = O.z_table(5, 3, 77)
    for u in range(5):
        for j in range(1, 4):
            assert int(z[u, j - 1]) == O.keyed_hash(77, ord("Z"), [u | (j << 32)])
    colour = np.array([0, 2, 1, 2, 0], dtype=np.uint8)
    motif = np.array([1, 0, 2], dtype=np.uint8)  # shades: colour0 -> {0}, colour2 -> {1,2}
    zm = O.z_table(5, 3, 77, colour=colour, n_colours=3, motif=motif)
    off = {0: 0, 1: 1, 2: 1}
    for u in range(5):
        s = int(colour[u])
        for j in range(1, 4):
            acc = 0
            for r_ in range(int(motif[s])):
                dd = off[s] + r_
                acc ^= O.gf_mul(O.keyed_hash(77, ord("G"), [u | (dd << 32)]),
                                O.keyed_hash(77, ord("W"), [dd | (j << 32)]))
            assert int(zm[u, j - 1]) == acc
    assert not zm[2].any()  # colour 1 has multiplicity 0


def _rand_case(seed):
    g = inputs.tiny_graph(seed, n_max=8, m_max=28, t_max=6)
    return g


def test_invariances(oracle_mod):
    O = oracle_mod
    r = random.Random(11)
    for gi in range(30):
        g = _rand_case(1000 + gi)
        k = r.randint(2, min(5, g.n))
        delta = r.randint(0, 3)
        seed = r.getrandbits(63)
        F = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed)
        # (i) permutation of the edge list
        p = np.random.default_rng(gi).permutation(g.m)
        assert O.sieve(g.n, g.src[p], g.dst[p], g.t[p], k, delta, seed) == F
        # (ii) duplicated triples
        s2, d2, t2 = (np.concatenate([a, a[: g.m // 2]]) for a in (g.src, g.dst, g.t))
        assert O.sieve(g.n, s2, d2, t2, k, delta, seed) == F
        # (iii) self-loops added / removed
        loops = np.arange(g.n, dtype=np.uint32)
        s3 = np.concatenate([g.src, loops])
        d3 = np.concatenate([g.dst, loops])
        t3 = np.concatenate([g.t, np.ones(g.n, dtype=np.uint32)])
        assert O.sieve(g.n, s3, d3, t3, k, delta, seed) == F
        keep = g.src != g.dst
        assert O.sieve(g.n, g.src[keep], g.dst[keep], g.t[keep], k, delta, seed) == F
        # (iv) delta beyond the time span saturates
        span = int(g.t.max() - g.t.min())
        assert O.sieve(g.n, g.src, g.dst, g.t, k, span, seed) == O.sieve(g.n, g.src, g.dst, g.t, k, span + 7, seed)
        # (v) equal timestamps: F independent of delta
        tt = np.full(g.m, 3, dtype=np.uint32)
        assert O.sieve(g.n, g.src, g.dst, tt, k, 0, seed) == O.sieve(g.n, g.src, g.dst, tt, k, 5, seed)
        # (vii) iteration-range split
        a = r.randint(0, 1 << k)
        Fa = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=0, it_end=a) if a else 0
        Fb = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, it_begin=a, it_end=1 << k) if a < (1 << k) else 0
        assert Fa ^ Fb == F
        F2_, per = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, per_iteration=True)
        assert F2_ == F and int(np.bitwise_xor.reduce(per)) == F
        assert per[0] == 0  # L = empty set: z^L = 0


def test_motif_colour_exclusion(oracle_mod):
    """(vi) Vertices whose colour is absent from M have z = 0, so removing
    them and their edges (the preprocessing of Sec. 5.1) leaves F unchanged."""
    O = oracle_mod
    r = random.Random(12)
    for gi in range(30):
        g = _rand_case(2000 + gi)
        k = r.randint(2, min(5, g.n))
        motif = inputs.random_motif(k, g.n_colours, np.random.default_rng(gi))
        delta = r.randint(0, 3)
        seed = r.getrandbits(63)
        kw = dict(colour=g.colour, n_colours=g.n_colours, motif=motif)
        F = O.sieve(g.n, g.src, g.dst, g.t, k, delta, seed, **kw)
        ok = (motif[g.colour[g.src]] > 0) & (motif[g.colour[g.dst]] > 0)
        assert O.sieve(g.n, g.src[ok], g.dst[ok], g.t[ok], k, delta, seed, **kw) == F


def test_yes_no_invariances(oracle_mod):
    """Monotone in delta; time reversal and vertex relabelling keep yes/no."""
    O = oracle_mod
    r = random.Random(13)
    for gi in range(30):
        g = _rand_case(3000 + gi)
        k = r.randint(2, min(5, g.n))
        prev = 0
        for delta in range(0, 5):
            c = O.count_paths(g.n, g.src, g.dst, g.t, k, delta)
            assert c >= prev
            prev = c
            yes = O.sieve(g.n, g.src, g.dst, g.t, k, delta, 5) != 0
            assert yes == (c > 0)
            tau = int(g.t.max())
            rev = O.sieve(g.n, g.dst, g.src, (tau + 1 - g.t).astype(np.uint32), k, delta, 6) != 0
            assert rev == yes
            perm = np.random.default_rng(gi).permutation(g.n).astype(np.uint32)
            rel = O.sieve(g.n, perm[g.src], perm[g.dst], g.t, k, delta, 7) != 0
            assert rel == yes


def test_rejects_invalid(oracle_mod):
    O = oracle_mod
    with pytest.raises(ValueError):
        O.sieve(3, [0], [1], [0], 3, 1, 1)  # timestamp 0
    with pytest.raises(ValueError):
        O.sieve(3, [0], [5], [1], 3, 1, 1)  # vertex out of range
    with pytest.raises(ValueError):
        O.sieve(3, [0], [1], [1], 3, 1, 1, colour=[0, 0, 0], n_colours=1, motif=[2])  # sum != k
