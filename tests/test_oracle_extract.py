"""Pins for the oracle's extraction of an optimal solution with k fine-grained
queries (Sec. 4.7), against what the paper and brute force fix:

* the section's figure (tests/golden): with M = {r, b, b, b} the only
  restless path with four vertices is v1 -> v4 -> v5 -> v6 (times 2, 3, 5);
  with M = {b, b, b, b} there is none;
* the figure of the fine-grained evaluation scheme: its highlighted path is
  the only one with four vertices;
* brute force on small random graphs (scalar and per-vertex resting times,
  colours and motifs, sources and targets): the extracted path is one of the
  restless paths a pure-Python enumeration finds under the same constraints,
  and its last timestamp is the least last timestamp among them; NO
  instances return None.
"""
import json
import os
import random

import numpy as np
import pytest

from test_oracle_sieve import F1, F2, F3, F4, py_paths, split

HERE = os.path.dirname(os.path.abspath(__file__))


def as_edges(path):
    verts, times = path
    return tuple((verts[j], verts[j + 1], times[j]) for j in range(len(times)))


def valid_paths(n, E, k, delta, colour=None, motif=None, sources=None, targets=None):
    out = []
    for p in py_paths(n, E, k, delta, colour=colour, motif=motif):
        if sources is not None and p[0][0] not in sources:
            continue
        if targets is not None and p[-1][1] not in targets:
            continue
        out.append(p)
    return out


def check_against_brute_force(O, n, E, k, delta, seed, colour=None, n_colours=0, motif=None, sources=None,
                              targets=None):
    s, d, t = split(E)
    got = O.extract(n, s, d, t, k, delta, seed, colour=colour, n_colours=n_colours, motif=motif, sources=sources,
                    targets=targets)
    want = valid_paths(n, E, k, delta, colour=colour, motif=motif, sources=sources, targets=targets)
    if not want:
        assert got is None
        return None
    assert got is not None
    assert len(got[0]) == k and len(got[1]) == k - 1
    p = as_edges(got)
    assert p in set(want), (p, want[:5])
    assert p[-1][2] == min(w[-1][2] for w in want)  # optimal: least largest timestamp
    return got


def test_figure_extraction(oracle_mod):
    O = oracle_mod
    fx = json.load(open(os.path.join(HERE, "golden", "fig_extraction.json")))
    n, E, delta, colour = fx["n"], fx["edges"], fx["delta"], fx["colour"]
    s, d, t = split(E)
    claim = fx["claims"][0]
    for seed in range(4):
        got = O.extract(n, s, d, t, claim["k"], delta, seed, colour=colour, n_colours=fx["n_colours"],
                        motif=claim["motif_count"])
        assert got == (claim["path"], [2, 3, 5])
        # every vertex black: no path agrees with M = {b, b, b, b}
        assert O.extract(n, s, d, t, 4, delta, seed, colour=colour, n_colours=2, motif=[0, 4]) is None
        # uncoloured: the highlighted path is the only one with four vertices
        assert O.extract(n, s, d, t, 4, delta, seed) == (claim["path"], [2, 3, 5])


def test_figure_fine_grained_path(oracle_mod):
    O = oracle_mod
    fx = json.load(open(os.path.join(HERE, "golden", "fig_fine_grained.json")))
    n, E, delta = fx["n"], fx["edges"], fx["delta"]
    s, d, t = split(E)
    claim = fx["claims"][0]
    for seed in range(3):
        assert O.extract(n, s, d, t, claim["k"], delta, seed) == (claim["path"], [2, 3, 5])
        assert O.extract(n, s, d, t, 5, delta, seed) is None


@pytest.mark.parametrize("E,n", [(F1, 8), (F2, 6), (F3, 7), (F4, 6)])
@pytest.mark.parametrize("delta", [0, 1, 2, 3])
def test_tiny_corpus_vs_brute_force(oracle_mod, E, n, delta):
    for k in range(2, 6):
        check_against_brute_force(oracle_mod, n, E, k, delta, seed=k + 7 * delta)


def random_graph(rng, n, m, tmax):
    E = set()
    while len(E) < m:
        a, b = rng.randrange(n), rng.randrange(n)
        if a != b:
            E.add((a, b, rng.randint(1, tmax)))
    return sorted(E)


def test_random_constraints_vs_brute_force(oracle_mod):
    rng = random.Random(2010)
    found = 0
    for case in range(60):
        n = rng.randint(4, 7)
        E = random_graph(rng, n, rng.randint(6, 11), rng.randint(3, 7))
        k = rng.randint(2, 5 if len(E) <= 9 else 4)
        delta = rng.randint(0, 3) if case % 2 else np.array([rng.randint(0, 3) for _ in range(n)], dtype=np.uint32)
        colour = motif = None
        n_colours = 0
        if case % 3 == 0:
            n_colours = 2
            colour = [rng.randrange(2) for _ in range(n)]
            r = rng.randint(0, k)
            motif = [r, k - r]
        sources = sorted(rng.sample(range(n), rng.randint(1, 2))) if case % 4 == 1 else None
        targets = sorted(rng.sample(range(n), rng.randint(1, 3))) if case % 5 == 2 else None
        got = check_against_brute_force(oracle_mod, n, E, k, delta, seed=case, colour=colour, n_colours=n_colours,
                                        motif=motif, sources=sources, targets=targets)
        found += got is not None
    assert found >= 20  # the sample holds YES instances, not only NO ones
