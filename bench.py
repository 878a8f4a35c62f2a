"""Benchmark: exact co-mining of the 36 three-edge temporal motifs on a
20M-edge power-law temporal graph (1M vertices, gamma 2.1, bursty timestamps
over 3e7 s, delta = 3600) on one MI355X.

One step = one full count of every motif over every root edge (the whole
search, device-resident graph and tree, counts copied back to the host).
Prints one JSON line with root edges/s, the speed-up over per-motif mining on
the same GPU, the HBM roofline position of the search kernel and the CPU
oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(st, time_bytes, n_roots):
    """Bytes the search must read once: each root's (src, dst, t); each
    per-vertex window's offset pair; one neighbour id per per-vertex window
    entry; (src, dst) per whole-list window entry; the time of each partial
    match kept for a deeper level.  Bisection probes are not counted."""
    return (n_roots * (8 + time_bytes) + st["win_list"] * 8 + st["ent_list"] * 4
            + st["ent_all"] * 8 + st["push"] * time_bytes)


def cpu_baseline(s, d, t, n, motifs, delta, target_s):
    import numpy as np
    import oracle
    og = oracle.OracleGraph(s, d, t, n)
    E = len(s)
    threads = oracle.max_threads()
    # calibrate on a small slice, then size the sample for ~target_s seconds
    probe = max(2000, E // 1000)
    r0 = E // 2
    t0 = time.perf_counter()
    for m in motifs:
        og.count(m, delta, roots=np.arange(r0, r0 + probe))
    dt = max(time.perf_counter() - t0, 1e-3)
    n_s = int(min(E - r0, max(probe, probe * target_s / dt)))
    roots = np.arange(r0, r0 + n_s)
    t0 = time.perf_counter()
    for m in motifs:
        og.count(m, delta, roots=roots)
    dt = time.perf_counter() - t0
    og.close()
    return {"value": n_s / dt, "unit": "root edges/s", "cores": threads, "kind": "oracle",
            "sample": "%d consecutive roots from the middle of the time order, all %d motifs, "
                      "one oracle pass per motif (%.1f s)" % (n_s, len(motifs), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (tests)")
    ap.add_argument("--per-motif-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--queues", type=int, default=0, help="root queues (0 = one per XCD)")
    ap.add_argument("--chunk", type=int, default=0, help="roots per queue grab (0 = default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the search shards by root time range with one "
              "count all-reduce, but multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2507_14813_amd import api, workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    t0 = time.perf_counter()
    wl = W.make_config(2, scale=args.scale)
    s, d, t, n = wl.graphs[0]
    motifs, delta = wl.motif_sets[0], wl.deltas[0]
    E = len(s)
    log("generated %d edges in %.1f s" % (E, time.perf_counter() - t0))

    g = api.Graph(s, d, t, n, sorted_by_t=True)
    tr = api.Tree(motifs, delta)
    gi, ti = g.info(), tr.info()
    stream = torch.cuda.current_stream()

    counts, st = api.count(g, tr, stats=True)
    algo_bytes = algorithmic_bytes(st, gi["time_bytes"], E)
    log("stats", st, "algorithmic bytes/launch %.3e" % algo_bytes)

    kw = dict(queues=args.queues, chunk=args.chunk)
    for _ in range(args.warmup):
        api.count(g, tr, **kw)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c, ms = api.count(g, tr, timed=True, **kw)
        kms.append(ms)
        if not np.array_equal(c, counts):
            raise SystemExit("counts changed between runs")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    value = E / (wall / args.steps)
    log("co-mine: %.3f ms/step wall, kernel %.3f ms avg" % (ms_step, sum(kms) / len(kms)))

    # per-motif mining on the same GPU: one launch per motif
    pm_ms, pm_wall = [], []
    for _ in range(args.per_motif_steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c, ms = api.count(g, tr, mode="per_motif", timed=True, **kw)
        torch.cuda.synchronize()
        pm_wall.append(time.perf_counter() - t1)
        pm_ms.append(ms)
        if not np.array_equal(c, counts):
            raise SystemExit("per-motif counts differ from co-mined counts")
    pm_step = sum(pm_wall) / len(pm_wall) if pm_wall else None
    if pm_wall:
        log("per-motif: %.3f ms/step wall, kernels %.3f ms"
            % (1e3 * pm_step, sum(pm_ms) / len(pm_ms)))

    k_avg_s = sum(kms) / len(kms) / 1e3
    achieved = algo_bytes / k_avg_s / 1e9
    out = {
        "metric": "root edges searched/s + co-mine speedup vs per-motif on GPU, exact counts",
        "value": value,
        "unit": "root edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/u32 (ids, times), u64 counts",
        "data": "synthetic",
        "config": {"workload": "powerlaw temporal graph V=%d E=%d gamma=2.1 span=3e7s "
                               "delta=%d; all 36 three-edge motifs on <=3 nodes (co-mined)"
                               % (n, E, delta),
                   "n_edges": E, "n_nodes": n, "delta": delta, "n_motifs": len(motifs),
                   "mg_tree_nodes": ti["n_nodes"], "similarity": round(ti["similarity"], 4)},
        "speedup_vs_per_motif": pm_step / (wall / args.steps) if pm_wall else None,
        "per_motif_root_edges_per_s": E / pm_step if pm_wall else None,
        "kernel_ms": sum(kms) / len(kms),
        "per_motif_kernel_ms": sum(pm_ms) / len(pm_ms) if pm_ms else None,
        "paper_context": "paper reports 2.4x (CPU, Xeon 8380) and 1.7x (GPU, A40) average "
                         "co-mining speedups on real graphs",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": algo_bytes},
        "stats": st,
        "total_matches": int(counts.sum()),
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(s, d, t, n, motifs, delta, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
