"""Benchmark: GF(2^64) sieve edge-updates per second on one MI355X.

One step = one full k-RestlessMotif query (all 2^k sieve iterations, levels
2..k, setup kernels and the final XOR) on the 10,000,000-edge Chung-Lu graph
(n=1,000,000, exponent 2.2, t in [1,10000] in 100 Gaussian bursts of sigma
20, 8 vertex colours), delta=20, a motif of k=10 colours, seed 3: the largest
single-query workload. The graph is resident in HBM before the timed region
starts. --workload path-scale times the 10^6-edge path query (k=8) instead.

An edge-update is one (edge, level l in 2..k, iteration L) triple, so a query
performs 2^k (k-1) m of them.

Prints one JSON line. Extra modes (not the driver's default):
  --mode batch   64 mixed queries on the same graph: one rs_run_batch vs 64 rs_run
  --mode serve   the continuous-batching server on four resident graphs vs
                 first-come first-served plain calls over the same arrivals
  --mode copy    a plain 1 GiB device copy, the reference for HBM byte counters
  --mode rows    random 512-byte row reads, writes and both (rs_probe_rows) over
                 an 8 GiB array: the practical ceiling of the prefix state's
                 access pattern
  --mode literal the literal reading of Eq. (poly-enc:1) (rs_run_literal) on
                 the 10^6-edge path query, against the VALU issue peak
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except Exception:  # noqa: BLE001
        return os.cpu_count() or 1


# Sources whose change invalidates the committed HBM counter figures of the
# level kernel (kernel code, launch shapes, defaults).
KERNEL_SOURCES = ("rs_device.h", "rs_level.h", "rs_kernels.hip", "rs_engine.hip", "rs_internal.h", "rs_compact.hip",
                  "rs_rrows.hip", "rs_group.hip")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_scan_chunglu_m1e6_k8_counters.md")
SQ_FILE = os.path.join(ROOT, "profiles", "k_scan_chunglu_m1e6_k8_sq.md")

# Plain-mode workloads: input generator, description, and the committed
# rocprofv3 summaries (HBM traffic, SQ issue rates) of their level kernel.
WORKLOADS = {
    "path-scale": ("config_path_scale",
                   "k-RestlessPath plain sieve, Chung-Lu(2.5) n=100000 m=1000000 t in [1,1000], delta=10, k=8 "
                   "(256 iterations), seed 2", COUNTERS_FILE, SQ_FILE),
    "motif-scale": ("config_motif_scale",
                    "k-RestlessMotif plain sieve, Chung-Lu(2.2) n=1000000 m=10000000, t in [1,10000] in 100 "
                    "Gaussian bursts (sigma 20), 8 colours, delta=20, motif of k=10 colours (1024 iterations), seed 3",
                    os.path.join(ROOT, "profiles", "k_scan_chunglu_m1e7_motif_k10_counters.md"),
                    os.path.join(ROOT, "profiles", "k_scan_chunglu_m1e7_motif_k10_sq.md")),
    "small": ("config_small",
              "k-RestlessPath plain sieve, uniform n=1000 m=10000 t in [1,100], delta=5, k=5 (32 iterations), seed 1",
              None, None),
}


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_08423_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_figures(path):
    """The `- key: value` lines of a committed rocprofv3 summary, if it was
    taken on the current kernel sources; else {}."""
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    fields[k.strip()] = v.strip().strip("`")
        return fields if fields.get("kernel-source-sha256") == kernel_source_hash() else {}
    except OSError:
        return {}


def committed_traffic(path=COUNTERS_FILE):
    """HBM bytes per level_scan launch from a committed counter summary."""
    if path is None:
        return None
    v = committed_figures(path).get("traffic-bytes-per-launch")
    return float(v) if v is not None else None


def _float(v):
    return float(v) if v is not None else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001
        pass
    return "unknown"


def cpu_baseline(g, q, m_dedup, budget_s=20.0):
    """The oracle (plain C, OpenMP over sieve iterations) on a bounded sample
    of the same query: a range of iterations starting at 1, sized to about
    budget_s. Returns the baseline record and the oracle's f_L over the range
    (for the bit-exact check against the GPU's values)."""
    import oracle

    cores = min(host_cores(), 64)
    kw = dict(colour=g.colour, n_colours=g.n_colours, motif=q.motif) if q.motif is not None else {}
    t0 = time.perf_counter()
    oracle.sieve(g.n, g.src, g.dst, g.t, q.k, q.delta, q.seed, it_begin=1, it_end=2, threads=1, **kw)
    one = max(time.perf_counter() - t0, 1e-3)
    n_it = int(max(1, min((1 << q.k) - 1, budget_s * cores / one)))
    n_it = max(cores, (n_it // cores) * cores) if n_it >= cores else n_it
    n_it = min(n_it, (1 << q.k) - 1)
    t0 = time.perf_counter()
    _, per = oracle.sieve(g.n, g.src, g.dst, g.t, q.k, q.delta, q.seed, it_begin=1, it_end=1 + n_it, threads=cores,
                          per_iteration=True, **kw)
    dt = time.perf_counter() - t0
    upd = n_it * (q.k - 1) * m_dedup
    rec = {"value": upd / dt, "unit": "edge-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"iterations [1,{1 + n_it}) of the {1 << q.k} of the same query ({n_it} sieve iterations, "
                     f"{dt:.1f} s, OpenMP over iterations on {cores} threads, {cpu_model()})"}
    return rec, 1, per


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "copy", "rows", "literal"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="--mode batch: the batched calls alone in the default shape (for kernel traces)")
    ap.add_argument("--workload", default="motif-scale", choices=sorted(WORKLOADS),
                    help="plain mode: the query timed (default: the 10^7-edge motif query)")
    # serve mode: offered load, arrival window, wall-clock cap, server budget
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--window", type=float, default=60.0)
    ap.add_argument("--cap", type=float, default=75.0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--group-updates", type=float, default=0, help="group work cap (0: the library default)")
    ap.add_argument("--streams", type=int, default=0)
    ap.add_argument("--sizes", default="10000,100000,1000000,10000000", help="edge counts of the served graphs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the sieve shards over iteration "
                                   "ranges across GPUs by design but no multi-GPU path is built"}))
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch

    import paper_2010_08423_amd as R
    from paper_2010_08423_amd import inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.mode == "copy":
        # calibration for HBM byte counters: a plain device copy of known size
        n = 1 << 30
        x = torch.ones(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": n, "bytes_written_per_copy": n,
                          "copies": args.steps}), flush=True)
        return
    if args.mode == "rows":
        # the prefix state's access pattern on its own: whole 512-byte rows at
        # random rows of an array far larger than the caches
        n_rows = 1 << 24
        rows = torch.zeros((n_rows, 64), dtype=torch.int64, device="cuda")
        steps, per_step = 128, {0: 16, 1: 16, 2: 24}
        res = {}
        for mode, name in ((0, "read"), (1, "write"), (2, "read2_write1")):
            best = None
            for waves in (4096, 8192):
                out = torch.empty((waves, 64), dtype=torch.int64, device="cuda")
                R.probe_rows(rows, out, waves, 4, mode)  # warm-up
                times = []
                for _ in range(max(args.steps // 4, 3)):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    R.probe_rows(rows, out, waves, steps, mode)
                    b.record()
                    b.synchronize()
                    times.append(a.elapsed_time(b))
                ms = sorted(times)[len(times) // 2]
                gbps = waves * steps * per_step[mode] * 512 / (ms * 1e-3) / 1e9
                if best is None or gbps > best["GBps"]:
                    best = {"GBps": gbps, "waves": waves, "ms": ms}
            res[name] = best
        print(json.dumps({"mode": "rows", "row_bytes": 512, "array_bytes": n_rows * 512, "rows_per_step": per_step,
                          "steps": steps, "results": res}), flush=True)
        return
    if args.mode != "plain":
        from paper_2010_08423_amd import bench_modes

        out = bench_modes.run(args)
        print(json.dumps(out), flush=True)
        return

    gen, desc, counters_file, sq_file = WORKLOADS[args.workload]
    log("generating graph")
    g, q = getattr(inputs, gen)()
    gd = R.Graph.from_inputs(g)
    info = gd.info()
    m = info["m"]
    upd = (1 << q.k) * (q.k - 1) * m
    # Kernel timing is on from the warmup on, so the one-off measurement of the
    # window counts (used for the byte accounting) happens before the timed region.
    R.profile_enable(True)
    for _ in range(max(args.warmup, 1)):
        r = R.run(gd, q.k, q.delta, q.seed, motif=q.motif)
    F = r.fingerprint

    # Timed region: K full queries, kernel timing live on the launch stream.
    R.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = R.run(gd, q.k, q.delta, q.seed, motif=q.motif)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    R.profile_enable(False)
    if F is not None and r.fingerprint != F:
        raise SystemExit("fingerprint changed between runs")
    ms = dt * 1e3 / args.steps
    n_scan, ms_scan, bytes_scan = R.profile_get("level_scan")
    avg_scan_ms = ms_scan / max(n_scan, 1)
    # Algorithmic bytes of one launch: the method's per-unit figure (per
    # edge-update of levels 3..k-1, two 8-byte window reads and one 8-byte
    # state write) over the edge-updates the launch performs. The exact
    # computation skips edges whose window is empty or whose product reaches
    # no read slot, and stores only read slots, so per 64-iteration chunk it
    # moves 1024 B per gathered edge and 512 B per stored slot, plus the
    # per-edge indices, flags and product rows once per launch (counts
    # measured by the library; the byte sum comes with the kernel timing).
    alg_bytes = bytes_scan / max(n_scan, 1)
    achieved = alg_bytes / (avg_scan_ms * 1e-3) / 1e9
    # The same per-unit figure over all 2^k (k-1) m nominal edge-updates,
    # i.e. the bytes a dense evaluation of the levels would move; its rate
    # exceeds the HBM peak because the skipped updates are never done.
    kq = (q.k + 3) // 4 * 4
    # chunks per launch, from the launches counted: levels 4..k-1 (level 2 is
    # folded into level 3 at k >= 4, which has a class of its own) once per
    # group of chunks
    chunks = max(1, (1 << q.k) // 64)
    per_query = n_scan / max(args.steps, 1)
    groups = per_query / max(q.k - 4, 1) if q.k >= 5 else 1
    chunks_per_launch = max(1, round(chunks / max(groups, 1)))
    dense_bytes = (1536.0 * chunks_per_launch + 12 + 8 * kq) * m
    dense = dense_bytes / (avg_scan_ms * 1e-3) / 1e9
    classes = {}
    for c in ("level_scan", "level_first", "level_top", "qtable", "ztable", "window"):
        n, tot, b = R.profile_get(c)
        classes[c] = {"launches": n, "avg_ms": tot / max(n, 1), "GBps": b / max(tot, 1e-9) / 1e6}
    out = {
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
        "config": {"workload": desc,
                   "n": info["n"], "m": m, "k": q.k, "delta": q.delta, "seed": q.seed,
                   "edge_updates_per_query": upd, "fingerprint": f"{r.fingerprint:#018x}"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": committed_traffic(counters_file),
                     "kernel": f"k_scan<kq={kq},E=16>, prefix levels 4..k-1, {chunks_per_launch} chunks per launch",
                     "avg_launch_ms": avg_scan_ms, "launches": n_scan,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     # the dense evaluation's bytes at the same per-unit figure, and their rate
                     "dense_equivalent_bytes_per_launch": dense_bytes, "dense_equivalent_GBps": dense,
                     # issue rates of the same kernel from the committed SQ counter summary
                     "valu_frac": _float(committed_figures(sq_file).get("valu-frac")) if sq_file else None,
                     "salu_frac": _float(committed_figures(sq_file).get("salu-frac")) if sq_file else None},
        "kernels": classes,
    }
    # look-back events of one more (untimed) query: predecessor runs
    # recomputed after the bounded wait, probe rounds that found no record
    R.lookback_count(True)
    rl = R.run(gd, q.k, q.delta, q.seed, motif=q.motif)
    lb = R.lookback_get()
    R.lookback_count(False)
    if rl.fingerprint != F:
        raise SystemExit("fingerprint changed with look-back counting on")
    out["lookback_one_query"] = {"recomputed_predecessor_runs": lb[0], "unanswered_probe_rounds": lb[1]}
    exact = True
    if rank == 0 and not args.no_cpu_baseline:
        rec, a, per = cpu_baseline(g, q, m)
        out["cpu_baseline"] = rec
        # bit-exact check outside the timed region: the GPU's f_L over the
        # oracle's sample range of the same query. The GPU runs the whole
        # 128-iteration blocks holding that range, so that the last level
        # takes its chunk-pair form as in the timed query.
        b0 = (a // 128) * 128
        b1 = min(1 << q.k, -(-(a + len(per)) // 128) * 128)
        rg = R.run(gd, q.k, q.delta, q.seed, motif=q.motif, it_begin=b0, it_end=b1, per_iteration=True)
        got = rg.per_iteration[a - b0:a - b0 + len(per)]
        exact = [int(x) for x in got] == [int(x) for x in per]
        out["bit_exact"] = exact
        out["bit_exact_sample"] = (f"f_L of iterations [{a},{a + len(per)}) on the GPU (run over [{b0},{b1})) "
                                   f"vs the oracle")
    print(json.dumps(out), flush=True)
    if not exact:
        raise SystemExit("GPU per-iteration values differ from the oracle's")


if __name__ == "__main__":
    main()
