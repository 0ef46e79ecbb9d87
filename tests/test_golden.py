"""The paper's worked examples (tests/golden/*.json, each citing its figure):
the highlighted paths are restless paths of the printed graphs, the sieve
says YES for them, and the walk-but-no-path example says NO."""
import glob
import itertools
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURES = sorted(glob.glob(os.path.join(HERE, "golden", "fig_*.json")))


def load(path):
    with open(path) as f:
        return json.load(f)


def is_restless_path(edges, path, delta):
    es = set(map(tuple, edges))
    times = []
    for a, b in zip(path, path[1:]):
        cands = sorted(t for (x, y, t) in es if x == a and y == b)
        if not cands:
            return False
        times.append(cands)
    # choose times greedily is not enough in general; search all combinations
    def rec(i, last):
        if i == len(times):
            return True
        for t in times[i]:
            if i == 0 or (0 <= t - last <= delta):
                if rec(i + 1, t):
                    return True
        return False

    return len(set(path)) == len(path) and rec(0, None)


@pytest.mark.parametrize("path", FIXTURES, ids=[os.path.basename(p) for p in FIXTURES])
def test_fixture_claims(oracle_mod, path):
    O = oracle_mod
    fx = load(path)
    assert fx["citation"]
    n, E, delta = fx["n"], fx["edges"], fx["delta"]
    s = [e[0] for e in E]
    d = [e[1] for e in E]
    t = [e[2] for e in E]
    for c in fx["claims"]:
        if "path" in c:
            assert is_restless_path(E, c["path"], delta) == c["yes"]
            kw = {}
            if "motif_count" in c:
                kw = dict(colour=fx["colour"], n_colours=fx["n_colours"], motif=c["motif_count"])
            k = c["k"]
            assert O.count_paths(n, s, d, t, k, delta, **kw) >= 1
            for seed in range(5):
                assert O.sieve(n, s, d, t, k, delta, seed, **kw) != 0
        else:
            # no restless path from source to dest of any length
            src_v, dst_v = c["source"], c["dest"]
            reach = False
            for k in range(2, n + 1):
                # restless paths from src_v to dst_v with k vertices
                for mid in itertools.permutations([v for v in range(n) if v not in (src_v, dst_v)], k - 2):
                    if is_restless_path(E, [src_v, *mid, dst_v], delta):
                        reach = True
            assert reach == c["yes"]
    if "walk" in fx:
        w = fx["walk"]
        es = set(map(tuple, E))
        last = None
        for a, b in zip(w, w[1:]):
            ts = [tt for (x, y, tt) in es if x == a and y == b]
            assert len(ts) == 1
            if last is not None:
                assert 0 <= ts[0] - last <= delta
            last = ts[0]
        # the walk has len(w) vertex visits; with that many (and one fewer)
        # vertices there is no restless path anywhere, so the sieve must
        # cancel every walk and return 0
        for k in (len(w) - 1, len(w)):
            assert O.count_paths(n, s, d, t, k, delta) == 0
            for seed in range(20):
                assert O.sieve(n, s, d, t, k, delta, seed) == 0
    if "motif_claim" in fx:
        mc = fx["motif_claim"]
        motif = np.bincount(mc["motif_colours"], minlength=mc["n_colours"]).astype(np.uint8)
        assert is_restless_path(E, mc["path"], delta)
        kw = dict(colour=mc["colour"], n_colours=mc["n_colours"], motif=motif)
        assert O.count_paths(n, s, d, t, mc["k"], delta, **kw) >= 1
        for seed in range(5):
            assert O.sieve(n, s, d, t, mc["k"], delta, seed, **kw) != 0
