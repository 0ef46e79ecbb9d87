"""The batched, served and literal-reading benchmark modes of bench.py.

batch: 64 queries on the 1,000,000-edge Chung-Lu graph (k uniform in 4..12,
       delta uniform in 2..50, half path and half motif over 8 colours, seeds
       100..163), launch shape chosen by the autotuner on a sample of the mix.
       A step is one rs_run_batch of all 64; the comparison is the same 64
       queries as 64 plain rs_run calls one after another. Fingerprints must
       agree exactly.
serve: resident graphs (by default the served set m = 1e4, 1e5, 1e6, 1e7,
       alternately uniform and Chung-Lu),
       open-loop Poisson arrivals (k uniform in 4..12, delta in 1..100, 30 %
       motif queries over 8 colours) submitted at their arrival times to the
       continuous-batching server; the comparison serves the same arrivals
       first-come first-served with plain rs_run calls. Both runs stop at the
       same wall-clock cap; what has not completed by then is counted, not
       timed.
"""
from __future__ import annotations

import dataclasses
import threading
import time

import numpy as np

import paper_2010_08423_amd as R
from paper_2010_08423_amd import inputs


def _log(*a):
    import sys

    print(*a, file=sys.stderr, flush=True)


def _updates(m, q):
    span = (q.it_end - q.it_begin) if (q.it_begin or q.it_end) else (1 << q.k)
    return span * (q.k - 1) * m


def run_batch_mode(args):
    import torch

    _log("generating graph")
    g, _ = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    m = gd.info()["m"]
    qs = inputs.batch_mix()
    upd = sum(_updates(m, q) for q in qs)
    if getattr(args, "batch_only", False):
        return _batch_only(args, gd, qs, upd)
    # autotune on one query per k of the mix, each cut to its first four
    # 64-iteration chunks: every level structure of the mix is timed, and the
    # tuning time stays bounded
    by_k = {}
    for q in qs:
        by_k.setdefault(q.k, q)
    sample = [dataclasses.replace(q, it_begin=0, it_end=min(256, 1 << q.k)) for q in by_k.values()]
    _log("autotuning on", [(q.k, q.delta, q.it_end) for q in sample])
    t0 = time.perf_counter()
    R.autotune(gd, sample)
    # the batched shape on a batch like the real one: every query of the mix,
    # each cut to its first two chunks (many rounds, so the stream lanes overlap)
    bsample = [dataclasses.replace(q, it_begin=0, it_end=min(128, 1 << q.k)) for q in qs]
    tuned = R.autotune_batch(gd, bsample)
    tune_s = time.perf_counter() - t0
    # plain reference: one query at a time
    _log("plain: 64 queries one at a time")
    for q in qs[:2]:
        R.run(gd, q.k, q.delta, q.seed, motif=q.motif)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [R.run(gd, q.k, q.delta, q.seed, motif=q.motif).fingerprint for q in qs]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    _log(f"plain {plain_s:.2f} s")
    # batched
    graphs = [gd] * len(qs)
    for _ in range(args.warmup):
        res, st = R.run_batch(graphs, qs)
    R.profile_enable(True)
    R.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, st = R.run_batch(graphs, qs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    R.profile_enable(False)
    if st != R.RS_OK:
        raise SystemExit(f"rs_run_batch failed: {st}")
    got = [r.fingerprint for r in res]
    if got != plain:
        bad = [i for i in range(len(qs)) if got[i] != plain[i]]
        raise SystemExit(f"batched fingerprints differ from plain for queries {bad}")
    # look-back events of one more (untimed) batch on the four stream lanes,
    # whose rounds' waves are not guaranteed to be resident together
    R.lookback_count(True)
    res2, _ = R.run_batch(graphs, qs)
    lb_batch = R.lookback_get()
    R.lookback_count(False)
    if [r.fingerprint for r in res2] != plain:
        raise SystemExit("batched fingerprints changed with look-back counting on")
    return {
        "metric": "queries/s (batched vs plain, equal fingerprints)",
        "value": len(qs) / dt,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "64-query batch on Chung-Lu(2.5) n=100000 m=1000000 t in [1,1000]: k in 4..12, "
                               "delta in 2..50, half motif over 8 colours, seeds 100..163",
                   "edge_updates_per_step": upd,
                   "tuning": {"edges_per_tile": tuned.edges_per_tile, "waves_per_block": tuned.waves_per_block,
                              "top_edges_per_tile": tuned.top_edges_per_tile},
                   "autotune_s": tune_s},
        "batched": {"queries_per_s": len(qs) / dt, "edge_updates_per_s": upd / dt, "s_per_batch": dt},
        "plain": {"queries_per_s": len(qs) / plain_s, "edge_updates_per_s": upd / plain_s, "s_total": plain_s},
        "speedup_vs_plain": plain_s / dt,
        "fingerprints_equal": True,
        "lookback_one_batch": {"recomputed_predecessor_runs": lb_batch[0], "unanswered_probe_rounds": lb_batch[1]},
    }


def _batch_only(args, gd, qs, upd):
    """The batched calls alone, in the default launch shape (no autotuner, no
    plain reference): the run a kernel trace of the batched path profiles."""
    import torch

    graphs = [gd] * len(qs)
    for _ in range(args.warmup):
        R.run_batch(graphs, qs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res, st = R.run_batch(graphs, qs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if st != R.RS_OK:
        raise SystemExit(f"rs_run_batch failed: {st}")
    return {
        "metric": "queries/s (batched calls alone, default launch shape)",
        "value": len(qs) / dt,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "64-query batch on Chung-Lu(2.5) n=100000 m=1000000 t in [1,1000]: k in 4..12, "
                               "delta in 2..50, half motif over 8 colours, seeds 100..163",
                   "edge_updates_per_step": upd},
        "batched": {"queries_per_s": len(qs) / dt, "edge_updates_per_s": upd / dt, "s_per_batch": dt},
    }


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


def run_serve_mode(args):
    import torch

    rate, window, cap = args.rate, args.window, args.cap
    _log("generating served graphs")
    gs = inputs.served_graphs(sizes=tuple(int(x) for x in args.sizes.split(",")))
    gds = [R.Graph.from_inputs(g) for g in gs]
    ms = [gd.info()["m"] for gd in gds]
    stream = inputs.served_stream(rate, window, len(gs))
    _log(f"{len(stream)} arrivals over {window} s at {rate}/s")

    # served
    srv = R.Server(hbm_budget=int(args.budget_gb * (1 << 30)), group_edge_updates=int(args.group_updates),
                   streams=args.streams)
    ids = [srv.add_graph(gd) for gd in gds]
    tickets = [None] * len(stream)
    t_sub = [0.0] * len(stream)
    start = time.perf_counter()

    def submitter():
        for i, (ta, gi, q) in enumerate(stream):
            d = start + ta - time.perf_counter()
            if d > 0:
                time.sleep(d)
            t_sub[i] = time.perf_counter()
            tickets[i] = srv.submit(ids[gi], q)

    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    st_window = srv.stats()  # when the last arrival is in: the backlog the window leaves
    t_window = time.perf_counter() - start
    lat, fps, done = [], {}, 0
    _log(f"arrivals in after {t_window:.1f} s: {st_window['completed']} completed, "
         f"{st_window['queued'] + st_window['inflight']} waiting or running")
    for i, tk in enumerate(tickets):
        if i % 500 == 0:
            _log(f"collecting results: {i}/{len(tickets)} at {time.perf_counter() - start:.1f} s")
        left_ms = int(max(0.0, start + cap - time.perf_counter()) * 1e3)
        r = srv.poll(tk, wait_ms=left_ms) if left_ms > 0 else srv.poll(tk, wait_ms=0)
        if r is not None and r.status == R.RS_OK:
            fps[i] = r.fingerprint
    end_served = time.perf_counter()
    st = srv.stats()
    for i, tk in enumerate(tickets):
        if i not in fps:
            srv.cancel(tk)
    cancelled = srv.stats()["cancelled"]
    srv.close()
    served_elapsed = end_served - start
    p50, p99 = st["p50_ms"], st["p99_ms"]
    served_done = len(fps)
    done_updates = sum(_updates(ms[stream[i][1]], stream[i][2]) for i in fps)

    # plain first-come first-served over the same arrivals, same cap
    _log("plain FCFS over the same arrivals")
    torch.cuda.synchronize()
    start = time.perf_counter()
    plain_lat, plain_fp = [], {}
    next_log = 10.0
    for i, (ta, gi, q) in enumerate(stream):
        now = time.perf_counter()
        if now - start >= cap:
            break
        if now - start >= next_log:
            _log(f"plain: {i} arrivals handled at {now - start:.1f} s")
            next_log += 10.0
        if start + ta > now:
            time.sleep(start + ta - now)
        plain_fp[i] = R.run(gds[gi], q.k, q.delta, q.seed, motif=q.motif).fingerprint
        plain_lat.append((time.perf_counter() - (start + ta)) * 1e3)
    plain_elapsed = time.perf_counter() - start
    pp50, pp99 = _percentiles(plain_lat)
    common = [i for i in fps if i in plain_fp]
    mismatch = [i for i in common if fps[i] != plain_fp[i]]
    if mismatch:
        raise SystemExit(f"served fingerprints differ from plain for arrivals {mismatch[:10]}")
    return {
        "metric": "queries/s + p50/p99 latency (served vs plain FCFS, equal fingerprints)",
        "value": served_done / served_elapsed,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": served_elapsed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"served stream: Poisson {rate}/s for {window} s over 4 resident graphs "
                               f"(m = {ms}), k in 4..12, delta in 1..100, 30% motif; cap {cap} s",
                   "arrivals": len(stream), "hbm_budget_gb": args.budget_gb,
                   "group_edge_updates": args.group_updates or 4e9, "streams": args.streams or 2},
        "served": {"completed": served_done, "queries_per_s": served_done / served_elapsed,
                   "edge_updates_per_s": done_updates / served_elapsed, "p50_ms": p50, "p99_ms": p99,
                   "jobs": st["jobs"], "slices": st["slices"], "deferred": st["deferred"],
                   "held_gb": st["held_bytes"] / 2**30, "elapsed_s": served_elapsed,
                   # at the end of the arrival window: completed so far and the backlog left
                   "at_window_end": {"t_s": t_window, "completed": st_window["completed"],
                                     "backlog": st_window["queued"] + st_window["inflight"],
                                     "queued": st_window["queued"], "inflight": st_window["inflight"],
                                     "deferred": st_window["deferred"]},
                   # at the cap: what had not completed is cancelled
                   "backlog_at_cap": len(stream) - served_done, "cancelled_at_cap": cancelled},
        "plain": {"completed": len(plain_fp), "queries_per_s": len(plain_fp) / plain_elapsed,
                  "p50_ms": pp50, "p99_ms": pp99, "elapsed_s": plain_elapsed},
        "fingerprints_equal_on_common": len(common),
    }


# Wave64 VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction
# per SIMD every 4 clocks, i.e. 3.93e13 32-bit lane operations per second.
VALU_LANE_OPS_PEAK = 256 * 4 * 2.4e9 / 4 * 64
# VALU instructions per product of the literal level kernel, counted in its
# compiled gfx950 code: a window-term product (table of multiples of the
# wave-uniform y, 16-nibble comb, reduction) and a slot product (the slot's
# sum times z^L_u through a per-lane table, with the subset XOR of z_u).
LITERAL_VALU_PER_TERM = 111
LITERAL_VALU_PER_SLOT = 140


def literal_work(src, dst, t, n, k, delta, chunks):
    """Products of one literal-reading query on the canonical edge list, per
    level (the work the level kernel performs), as {level: (window-term
    products, slot products)} over all chunks: level 2 one term per edge of a
    slot some window reads, levels 3..k-1 one per window slot of such edges,
    level k one per window slot of every edge; one slot product per slot
    whose sum is formed (a read slot at levels below k; at levels >= 3 only
    if one of its edges has a non-empty window)."""
    m = len(dst)
    first = np.ones(m, bool)
    first[1:] = (dst[1:] != dst[:-1]) | (t[1:] != t[:-1])
    slot = np.cumsum(first) - 1
    ns = int(slot[-1]) + 1 if m else 0
    key = dst[first].astype(np.int64) * (1 << 32) + t[first].astype(np.int64)  # sorted slot keys
    d = np.full(n, int(delta), np.int64) if np.isscalar(delta) else np.asarray(delta, np.int64)
    ti = t.astype(np.int64)
    lo_t = np.maximum(ti - d[src], 1)
    lo = np.searchsorted(key, src.astype(np.int64) * (1 << 32) + lo_t, side="left")
    hi = np.searchsorted(key, src.astype(np.int64) * (1 << 32) + ti, side="right")
    win = hi - lo
    cover = np.zeros(ns + 1, np.int64)
    np.add.at(cover, lo, 1)
    np.add.at(cover, hi, -1)
    need = np.cumsum(cover)[:ns] > 0
    in_need = need[slot]
    fed = np.bincount(slot, weights=(win > 0), minlength=ns) > 0  # a slot with a non-empty window
    work = {}
    if k == 2:
        work[2] = (m, ns)
    else:
        work[2] = (int(in_need.sum()), int(need.sum()))
        for l in range(3, k):
            work[l] = (int(win[in_need].sum()), int((need & fed).sum()))
        work[k] = (int(win.sum()), int(fed.sum()))
    return {l: (a * chunks, b * chunks) for l, (a, b) in work.items()}


def run_literal_mode(args):
    """The literal reading of Eq. (poly-enc:1) (rs_run_literal) on the
    10^6-edge path query: whole queries timed, the level kernel's launches
    timed live, its window-term products counted on the host."""
    import torch

    _log("generating graph")
    g, q = inputs.config_path_scale()
    gd = R.Graph.from_inputs(g)
    info = gd.info()
    m = info["m"]
    upd = (1 << q.k) * (q.k - 1) * m
    R.profile_enable(True)
    for _ in range(max(args.warmup, 1)):
        r = R.run_literal(gd, q.k, q.delta, q.seed, slots=False)
    F = r.fingerprint
    R.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = R.run_literal(gd, q.k, q.delta, q.seed, slots=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_lvl, ms_lvl, _ = R.profile_get("literal_level")
    R.profile_enable(False)
    if r.fingerprint != F:
        raise SystemExit("slot checksum changed between runs")
    ms = dt * 1e3 / args.steps
    s, d, t = gd.edges()
    chunks = (1 << q.k) // 64
    work = literal_work(s, d, t, g.n, q.k, q.delta, chunks)
    terms_per_query = sum(a for a, _ in work.values())
    slots_per_query = sum(b for _, b in work.values())
    nominal_terms = (1 << q.k) * (q.k - 1) * m * (q.delta + 1)
    # every launch of the level kernel: one level of one group of chunks
    launches_per_query = n_lvl / max(args.steps, 1)
    # algorithmic VALU lane-operations of one query's products (each product
    # is one wave64 instruction stream over the 64 iterations of a chunk)
    lane_ops = 64 * (terms_per_query * LITERAL_VALU_PER_TERM + slots_per_query * LITERAL_VALU_PER_SLOT)
    achieved = lane_ops / (ms_lvl * 1e-3 / max(args.steps, 1)) / 1e12
    peak = VALU_LANE_OPS_PEAK / 1e12
    return {
        "metric": "GF(2^64) edge-updates/sec per sieve",
        "value": upd / (ms * 1e-3),
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "literal reading of Eq. (poly-enc:1) (y keyed by the predecessor's arrival time, "
                               "per-slot outputs), k-RestlessPath, Chung-Lu(2.5) n=100000 m=1000000 t in [1,1000], "
                               "delta=10, k=8 (256 iterations), seed 2",
                   "n": info["n"], "m": m, "k": q.k, "delta": q.delta, "seed": q.seed,
                   "edge_updates_per_query": upd, "slot_checksum": f"{r.fingerprint:#018x}",
                   "reached_vertices": int((r.reach != R.UNREACHED).sum())},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "k_lit_level (all levels; one launch per level and chunk group)",
                     "avg_launch_ms": ms_lvl / max(n_lvl, 1), "launches_per_query": launches_per_query,
                     "window_terms_per_query": terms_per_query, "slot_products_per_query": slots_per_query,
                     "products_per_level": {str(l): list(v) for l, v in work.items()},
                     "nominal_terms_per_query": nominal_terms,
                     "valu_ops_per_term": LITERAL_VALU_PER_TERM, "valu_ops_per_slot": LITERAL_VALU_PER_SLOT},
        "kernel_ms_per_query": ms_lvl / max(args.steps, 1),
    }


def run(args):
    if args.mode == "batch":
        return run_batch_mode(args)
    if args.mode == "literal":
        return run_literal_mode(args)
    return run_serve_mode(args)
