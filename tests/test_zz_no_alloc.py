"""GPU: rs_run_noalloc, the entry point whose query workspace lives in the
library's per-GPU scratch array, gives the fingerprints and per-iteration
values of rs_run_ex (and the oracle) on two calls in a row, the second on a
smaller graph, changes no device memory allocation, and rejects a query whose
workspace exceeds the array."""
import numpy as np
import pytest

import oracle
from paper_2010_08423_amd import inputs
from parity_util import say

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


def test_noalloc_matches_run_ex_twice_then_smaller():
    import torch

    g1, q1 = inputs.config_small()  # n = 1000, m = 10^4, k = 5, delta = 5
    g2 = inputs.add_colours(inputs.uniform_graph(300, 3000, 40, seed=61), 3, seed=61)
    gd1, gd2 = R.Graph.from_inputs(g1), R.Graph.from_inputs(g2)
    inputs.add_colours(g1, 4, seed=62)
    gd1c = R.Graph.from_inputs(g1)
    motif = np.array([2, 1, 1, 3], np.uint8)
    cases = [
        (gd1, g1, dict(k=q1.k, delta=q1.delta, seed=q1.seed)),       # 10^4 edges
        (gd2, g2, dict(k=4, delta=3, seed=7)),                       # smaller: 3000 edges, k = 4
        (gd1c, g1, dict(k=7, delta=2, seed=8, motif=motif)),         # motif, 2 chunks of 64 iterations
        (gd2, g2, dict(k=6, delta=1, seed=9, it_begin=5, it_end=40)),  # an iteration range
    ]
    want = []
    for gd, g, kw in cases:
        r = R.run(gd, per_iteration=True, **kw)
        okw = dict(colour=g.colour, n_colours=g.n_colours, motif=kw["motif"]) if "motif" in kw else {}
        F = oracle.sieve(g.n, g.src, g.dst, g.t, kw["k"], kw["delta"], kw["seed"], it_begin=kw.get("it_begin", 0),
                         it_end=kw.get("it_end", 0), **okw)
        assert r.fingerprint == F
        want.append(r)
    # the first call on the device finds the scratch array; measure after it
    say("[noalloc] first call")
    r0 = R.run_noalloc(cases[0][0], per_iteration=True, **cases[0][2])
    assert r0.fingerprint == want[0].fingerprint
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for rep in range(2):
        for i, (gd, g, kw) in enumerate(cases):
            say(f"[noalloc] rep {rep} case {i}: m = {g.m}, {kw}")
            r = R.run_noalloc(gd, per_iteration=True, **kw)
            assert r.status == R.RS_OK
            assert r.fingerprint == want[i].fingerprint, (rep, i)
            assert np.array_equal(r.per_iteration, want[i].per_iteration), (rep, i)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_noalloc_rejects_oversized_query():
    g, q = inputs.config_path_scale()  # 10^6 edges: about 1.1 GiB of prefix state per chunk
    gd = R.Graph.from_inputs(g)
    say("[noalloc] oversized query")
    with pytest.raises(R.RSError) as ei:
        R.run_noalloc(gd, q.k, q.delta, q.seed)
    assert ei.value.status == R.RS_ENOMEM
    assert "scratch" in str(ei.value)
    # the array is still usable afterwards
    g2, q2 = inputs.config_small()
    gd2 = R.Graph.from_inputs(g2)
    assert R.run_noalloc(gd2, q2.k, q2.delta, q2.seed).fingerprint == R.run(gd2, q2.k, q2.delta, q2.seed).fingerprint
