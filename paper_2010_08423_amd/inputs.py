"""Seeded synthetic temporal graphs and query workloads.

This module only draws inputs: graphs, vertex colours, colour multisets,
query mixes and arrival times. It holds none of the sieve's arithmetic, so the
GPU path and the CPU oracle can both be fed from it.

Workload shapes follow the paper's experiments (Sec. 5.2): directed temporal
graphs with uniform or power-law degrees and integer timestamps in [1, tau].
The paper's own generator (a configuration model from earlier work) and its
datasets are not reproduced; the graphs below stand in for them:

* uniform: (src, dst) uniform over ordered pairs with src != dst;
* Chung-Lu: vertex weights w_i proportional to (i+1)^(-1/(beta-1)) for degree
  exponent beta, src and dst drawn independently proportional to w;
* timestamps uniform in [1, tau], or clustered in Gaussian bursts.

Edges are resampled until m distinct (src, dst, t) triples exist; the
returned edge list keeps the order in which each triple was first drawn, so it
is not sorted.

Every stream is seeded separately: ``np.random.default_rng([seed, STREAM])``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

GRAPH, TIMES, COLOURS, MOTIF, WORKLOAD, ARRIVALS = range(6)


@dataclasses.dataclass
class TemporalGraph:
    n: int
    src: np.ndarray  # uint32 [m]
    dst: np.ndarray  # uint32 [m]
    t: np.ndarray  # uint32 [m]
    colour: np.ndarray | None = None  # uint8 [n]
    n_colours: int = 0
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def t_max(self) -> int:
        return int(self.t.max()) if self.m else 0


@dataclasses.dataclass
class Query:
    k: int
    delta: int
    seed: int
    motif: np.ndarray | None = None  # uint8 counts per colour, sum == k
    it_begin: int = 0
    it_end: int = 0

    @property
    def iterations(self) -> int:
        return (self.it_end - self.it_begin) if (self.it_begin or self.it_end) else (1 << self.k)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def _distinct_edges(n, m, t_max, seed, draw_pairs, draw_times, batch_factor=1.3):
    """Draw (src, dst, t) until m distinct triples with src != dst exist."""
    if n < 2 and m > 0:
        raise ValueError("need at least two vertices")
    if m > n * (n - 1) * t_max:
        raise ValueError("more edges requested than distinct triples exist")
    g = _rng(seed, GRAPH)
    gt = _rng(seed, TIMES)
    keys = np.zeros(0, dtype=np.uint64)
    order = np.zeros(0, dtype=np.int64)
    drawn = 0
    src_all, dst_all, t_all = [], [], []
    while True:
        need = m - keys.shape[0]
        if need <= 0:
            break
        b = max(int(need * batch_factor) + 16, 1024)
        s, d = draw_pairs(g, b)
        t = draw_times(gt, b)
        ok = s != d
        s, d, t = s[ok].astype(np.uint64), d[ok].astype(np.uint64), t[ok].astype(np.uint64)
        src_all.append(s)
        dst_all.append(d)
        t_all.append(t)
        key = (s * np.uint64(n) + d) * np.uint64(t_max + 1) + t
        allk = np.concatenate([keys, key])
        allo = np.concatenate([order, np.arange(drawn, drawn + key.shape[0], dtype=np.int64)])
        drawn += key.shape[0]
        uk, first = np.unique(allk, return_index=True)
        keys, order = uk, allo[first]
    src = np.concatenate(src_all)
    dst = np.concatenate(dst_all)
    t = np.concatenate(t_all)
    pick = np.sort(order)[:m]
    return (src[pick].astype(np.uint32), dst[pick].astype(np.uint32), t[pick].astype(np.uint32))


def uniform_times(t_max):
    return lambda g, b: g.integers(1, t_max + 1, size=b)


def burst_times(t_max, n_bursts, sigma, seed):
    centres = _rng(seed, TIMES + 100).uniform(1, t_max, size=n_bursts)

    def draw(g, b):
        c = centres[g.integers(0, n_bursts, size=b)]
        return np.clip(np.rint(g.normal(c, sigma)), 1, t_max).astype(np.int64)

    return draw


def uniform_graph(n, m, t_max, seed, name="uniform") -> TemporalGraph:
    def pairs(g, b):
        return g.integers(0, n, size=b), g.integers(0, n, size=b)

    s, d, t = _distinct_edges(n, m, t_max, seed, pairs, uniform_times(t_max))
    return TemporalGraph(n=n, src=s, dst=d, t=t, name=name)


def chung_lu_weights(n, exponent):
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (exponent - 1.0))
    return w / w.sum()


def chung_lu_graph(n, m, exponent, t_max, seed, times=None, name="chung-lu") -> TemporalGraph:
    cdf = np.cumsum(chung_lu_weights(n, exponent))
    cdf[-1] = 1.0

    def pairs(g, b):
        s = np.searchsorted(cdf, g.random(b), side="right")
        d = np.searchsorted(cdf, g.random(b), side="right")
        return np.minimum(s, n - 1), np.minimum(d, n - 1)

    s, d, t = _distinct_edges(n, m, t_max, seed, pairs, times or uniform_times(t_max))
    return TemporalGraph(n=n, src=s, dst=d, t=t, name=name)


def add_colours(g: TemporalGraph, n_colours: int, seed: int) -> TemporalGraph:
    g.colour = _rng(seed, COLOURS).integers(0, n_colours, size=g.n).astype(np.uint8)
    g.n_colours = n_colours
    return g


def random_motif(k, n_colours, rng) -> np.ndarray:
    """Colour multiset of k i.i.d. uniform draws, as counts per colour."""
    draws = rng.integers(0, n_colours, size=k)
    return np.bincount(draws, minlength=n_colours).astype(np.uint8)


# --- the benchmark workloads -------------------------------------------------

def config_small():
    """Uniform directed temporal graph, n=1,000, m=10,000, t in [1,100];
    path query delta=5, k=5, seed 1."""
    g = uniform_graph(1000, 10_000, 100, seed=1, name="uniform n=1e3 m=1e4 tau=100")
    return g, Query(k=5, delta=5, seed=1)


def config_path_scale():
    """Chung-Lu exponent 2.5, n=100,000, m=1,000,000, t in [1,1000]; 8 colours
    (used by the batched mix); path query delta=10, k=8, seed 2."""
    g = chung_lu_graph(100_000, 1_000_000, 2.5, 1000, seed=2, name="chung-lu(2.5) n=1e5 m=1e6 tau=1000")
    add_colours(g, 8, seed=2)
    return g, Query(k=8, delta=10, seed=2)


def config_motif_scale():
    """Chung-Lu exponent 2.2, n=1,000,000, m=10,000,000, t in [1,10000] in
    100 Gaussian bursts (sigma 20); 8 colours; motif of k=10 i.i.d. colours,
    delta=20, seed 3."""
    times = burst_times(10_000, 100, 20.0, seed=3)
    g = chung_lu_graph(1_000_000, 10_000_000, 2.2, 10_000, seed=3, times=times,
                       name="chung-lu(2.2) n=1e6 m=1e7 tau=1e4 bursts")
    add_colours(g, 8, seed=3)
    motif = random_motif(10, 8, _rng(3, MOTIF))
    return g, Query(k=10, delta=20, seed=3, motif=motif)


def batch_mix(n_queries=64, n_colours=8, seed=4, k_range=(4, 12), delta_range=(2, 50)):
    """Query q: seed 100+q, k ~ U{4..12}, delta ~ U{2..50}; even q path, odd q
    motif over n_colours colours (k i.i.d. draws)."""
    r = _rng(seed, WORKLOAD)
    out = []
    for q in range(n_queries):
        k = int(r.integers(k_range[0], k_range[1] + 1))
        d = int(r.integers(delta_range[0], delta_range[1] + 1))
        motif = random_motif(k, n_colours, r) if q % 2 else None
        out.append(Query(k=k, delta=d, seed=100 + q, motif=motif))
    return out


def served_graphs(sizes=(10_000, 100_000, 1_000_000, 10_000_000), n_colours=8, seed=10):
    """Resident graphs of the served stream: alternately uniform and Chung-Lu
    (exponent 2.5), m edges, n = m/10 vertices, timestamps in [1, m/100],
    n_colours vertex colours."""
    out = []
    for i, m in enumerate(sizes):
        n, tau = max(m // 10, 2), max(m // 100, 1)
        if i % 2 == 0:
            g = uniform_graph(n, m, tau, seed=seed + i, name=f"uniform n={n} m={m} tau={tau}")
        else:
            g = chung_lu_graph(n, m, 2.5, tau, seed=seed + i, name=f"chung-lu(2.5) n={n} m={m} tau={tau}")
        out.append(add_colours(g, n_colours, seed=seed + i))
    return out


def served_stream(rate_per_s, duration_s, n_graphs, seed=5, k_range=(4, 12), delta_range=(1, 100),
                  motif_frac=0.3, n_colours=8):
    """Open-loop Poisson arrivals: list of (arrival_s, graph_index, Query)."""
    ra = _rng(seed, ARRIVALS)
    rw = _rng(seed, WORKLOAD)
    out = []
    tnow = 0.0
    i = 0
    while True:
        tnow += float(ra.exponential(1.0 / rate_per_s))
        if tnow >= duration_s:
            break
        gi = int(rw.integers(0, n_graphs))
        k = int(rw.integers(k_range[0], k_range[1] + 1))
        d = int(rw.integers(delta_range[0], delta_range[1] + 1))
        motif = random_motif(k, n_colours, rw) if rw.random() < motif_frac else None
        out.append((tnow, gi, Query(k=k, delta=d, seed=1000 + i, motif=motif)))
        i += 1
    return out


def tiny_graph(seed, n_max=8, m_max=30, t_max=6, n_colours=3):
    """Random tiny multigraph corpus entry (duplicates and self-loops kept on
    purpose: both are valid inputs)."""
    r = _rng(seed, GRAPH)
    n = int(r.integers(2, n_max + 1))
    m = int(r.integers(1, m_max + 1))
    src = r.integers(0, n, size=m).astype(np.uint32)
    dst = r.integers(0, n, size=m).astype(np.uint32)
    t = r.integers(1, t_max + 1, size=m).astype(np.uint32)
    colour = r.integers(0, n_colours, size=n).astype(np.uint8)
    return TemporalGraph(n=n, src=src, dst=dst, t=t, colour=colour, n_colours=n_colours, name=f"tiny-{seed}")
