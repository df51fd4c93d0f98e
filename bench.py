"""Benchmark of the grid KNN self-join on one MI355X.

A step is one pass of the whole hot path over the workload: for every dataset
of the workload, knn_build_index_device (bounds, eps sampling) and, for every
K, knn_self_join_device (grid levels, density-ordered persistent search,
failure re-queue and re-index), with the coordinates already resident in
device memory.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (description, [(dataset name, K list)])
    "expo_2m": ("skewed density: exponential(rate 40) coordinates, N=2e6, 2-D and 4-D, "
                "K in {1,8,32,64}", [("expo2d_2m", [1, 8, 32, 64]), ("expo4d_2m", [1, 8, 32, 64])]),
    "expo2d_2m_k32": ("exponential(rate 40) 2-D, N=2e6, K=32", [("expo2d_2m", [32])]),
    "unif2d_50k": ("uniform [0,100)^2, N=5e4, K=5", [("unif2d_50k", [5])]),
    "unif6d_5m": ("uniform [0,100)^6, N=5e6, K=32", [("unif6d_5m", [32])]),
    "clustered2d_20m": ("clustered catalogue-shaped 2-D, N=2e7, K=16", [("clustered2d_20m", [16])]),
}

HBM_PEAK_GBS = 8000.0
# FP64 vector peak without FMA: 256 CUs x 64 lanes x 2.4 GHz (78.6 TFLOP/s counts an FMA as 2)
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def alg_bytes(stats, n, K):
    """Algorithmic HBM bytes of the search kernel (k_search) over one join:
    per query it searched, its own coordinates (8n) and cell/row metadata (8),
    plus the output row (12K: int32 id + fp64 distance per neighbour) when it
    succeeds or its id (4) when it fails.  Queries handed to the heavy-query
    kernel, and queries deferred to the next level before the search, are not
    k_search's."""
    total = 0
    for L, (a, f) in enumerate(zip(stats["attempted"], stats["failed"])):
        h, hf = stats["heavy_queries"][L], stats["heavy_failed"][L]
        d = stats["deferred"][L]
        a, f = a - h - d, f - hf - d
        total += a * (8 * n + 8) + (a - f) * 12 * K + f * 4
    return total


def alg_ops(stats, n):
    """Algorithmic FP64 operations of k_search over one join: per candidate of
    the 3^n cells of every query it searched, n subtractions, n
    multiplications, n-1 additions and one comparison (3n).  The mean
    candidate count is over the queries searched (not deferred)."""
    return sum(((a - d) * c - hc) * 3 * n for a, d, c, hc in
               zip(stats["attempted"], stats["deferred"], stats["cand_per_query"],
                   stats["heavy_cand"]))


def kernel_source_hash():
    """sha256 of the search kernel's source: a traffic figure is reported only
    for the kernel it was measured on."""
    import hashlib
    src = os.path.join(ROOT, "paper_1810_04758_amd", "csrc", "search.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload):
    """HBM bytes per search launch from the committed counter summary of this
    workload (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by a copy kernel of
    known size); None when absent or taken on another version of the kernel."""
    path = os.path.join(ROOT, "profiles", f"k_search_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("search.hip sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(datasets, cases, budget_s=12.0):
    """Time the CPU oracle (as it stands) on a bounded sample of the same
    queries: a probe sizes the per-case sample so the whole leg takes about
    budget_s seconds of wall time on all host cores."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(0)
    name0, K0 = cases[0]
    probe = rng.choice(datasets[name0].shape[0], size=threads, replace=False)
    t0 = time.perf_counter()
    oracle.knn(datasets[name0], K0, rows=probe, threads=threads)
    per_query = (time.perf_counter() - t0) / threads
    per_case = int(max(threads, min(20000, budget_s / len(cases) / max(per_query, 1e-9))))
    per_case = (per_case // threads) * threads
    done = 0
    t_total = 0.0
    sample_desc = []
    for name, K in cases:
        D = datasets[name]
        rows = rng.choice(D.shape[0], size=min(per_case, D.shape[0]), replace=False)
        t0 = time.perf_counter()
        oracle.knn(D, K, rows=rows, threads=threads)
        t_total += time.perf_counter() - t0
        done += rows.shape[0]
        sample_desc.append(f"{name}/K={K}:{rows.shape[0]}q")
    return {"value": round(done / t_total, 2), "unit": "queries/s", "cores": threads,
            "kind": "oracle",
            "sample": "brute-force oracle on random rows of the same inputs: " +
                      ", ".join(sample_desc) + f" ({done} queries, {t_total:.1f} s wall)"}


def serving_leg(api, seconds, rate=200.0, budget_gib=96, inflight=4):
    """The serving workload: a Poisson stream (mean `rate` requests/s for
    `seconds`) of self-join requests over 24 resident datasets (N log-uniform
    in [1e4, 1e7], dims in {2,3,4,6}, uniform or exponential coordinates, K in
    {1,4,16,64}), admitted by device-memory footprint and run concurrently.
    Latency is submit -> results ready; most requests are latency-only
    (results discarded on the device), every 25th is copied back and compared
    with a solo join of the same index and K."""
    from paper_1810_04758_amd import datagen
    t_build = time.perf_counter()
    pool = datagen.serving_pool()
    idxs = [api.build_index(D) for D, _ in pool]
    t_build = time.perf_counter() - t_build
    arrivals, ds, ks = datagen.serving_trace(seconds, rate, len(pool))
    srv = api.Server(mem_budget_bytes=budget_gib << 30, max_inflight=inflight)
    for ix in idxs:
        srv.add_dataset(ix)
    checks = []
    tickets = []
    t0 = time.perf_counter()
    for i, (ta, d, k) in enumerate(zip(arrivals, ds, ks)):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        N = pool[d][0].shape[0]
        keep = (i % 25 == 0) and N <= 1_000_000
        tickets.append((srv.submit(int(d), int(k), N, discard=not keep), int(d), int(k), keep))
    for t, d, k, keep in tickets:
        ids, dists = srv.wait(t)
        if keep:
            checks.append((d, k, ids, dists))
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    same = True
    for d, k, ids, dists in checks:
        ref_i, ref_d = idxs[d].self_join_host(k)
        same = same and bool((ref_i == ids).all() and (ref_d == dists).all())
    for ix in idxs:
        ix.close()
    return {"requests": int(st["completed"]), "trace_seconds": seconds, "rate_per_s": rate,
            "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
            "mean_ms": round(st["mean_ms"], 2), "queries_per_s": round(st["queries_per_s"], 1),
            "requests_per_s": round(st["requests_per_s"], 2), "wall_s": round(wall, 2),
            "peak_inflight": int(st["peak_inflight"]), "peak_bytes": int(st["peak_bytes"]),
            "mix_equals_solo_checked": len(checks), "mix_equals_solo": same,
            "index_build_s": round(t_build, 2),
            "datasets": [desc for _, desc in pool]}


def schedule_comparison(api, dev, plan, outs, stream, reps=3):
    """The persistent schedule (device work queues per XCD, density-ordered
    items, heavy queries on workgroups of their own) against the plain one:
    one launch per level over every unsolved query in cell order, one work
    item per wavefront, no queue (same cell sides and lanes per query, so the
    same candidates are scanned).  Untimed by the step clock; best of `reps`
    joins each; search time (both search kernels) from the join's HIP events."""
    res = []
    tot = {0: [0.0, 0.0], 1: [0.0, 0.0]}
    for name, Ks in plan:
        idx = api.build_index(dev[name], stream=stream)
        for K in Ks:
            ids, dists = outs[(name, K)]
            row = dict(dataset=name, K=K)
            for sched in (0, 1):
                best_s = best_t = float("inf")
                # plain: no queue, no density order, no heavy-query workgroups
                extra = dict(schedule=1, heavy_min=-1) if sched else {}
                for _ in range(reps):
                    _, _, st = idx.self_join(K, ids=ids, dists=dists, stream=stream,
                                             with_stats=True, **extra)
                    best_s = min(best_s, sum(st["ms_search"]) + sum(st["ms_heavy"]))
                    best_t = min(best_t, st["ms_total"])
                key = "persistent" if sched == 0 else "plain"
                row[f"ms_search_{key}"] = round(best_s, 3)
                row[f"ms_join_{key}"] = round(best_t, 3)
                tot[sched][0] += best_s
                tot[sched][1] += best_t
            row["search_speedup"] = round(row["ms_search_plain"] / row["ms_search_persistent"], 3)
            res.append(row)
        idx.close()
    return {"cases": res,
            "search_speedup": round(tot[1][0] / tot[0][0], 3),
            "join_speedup": round(tot[1][1] / tot[0][1], 3)}


def graph_comparison(api, dev, plan, outs, stream, reps=3):
    """Eager joins against replays of the join captured in a HIP graph
    (use_graph): same index, K and outputs; wall time from submit to the
    stream being drained, best of `reps` each."""
    import torch
    res = []
    tot_e = tot_g = 0.0
    for name, Ks in plan:
        idx = api.build_index(dev[name], stream=stream)
        for K in Ks:
            ids, dists = outs[(name, K)]
            best = {}
            for mode in (0, 1):
                if mode:
                    idx.self_join(K, ids=ids, dists=dists, stream=stream, use_graph=1)  # capture
                b = float("inf")
                for _ in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    idx.self_join(K, ids=ids, dists=dists, stream=stream, use_graph=mode)
                    torch.cuda.synchronize()
                    b = min(b, (time.perf_counter() - t0) * 1e3)
                best[mode] = b
            tot_e += best[0]
            tot_g += best[1]
            res.append(dict(dataset=name, K=K, ms_eager=round(best[0], 3),
                            ms_graph_replay=round(best[1], 3),
                            speedup=round(best[0] / best[1], 3)))
        idx.close()
    return {"cases": res, "speedup": round(tot_e / tot_g, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="expo_2m", choices=sorted(WORKLOADS))
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--w-factor", type=float, default=0.0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the (untimed) knn_autotune pass before the timed steps")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="length of the serving trace (0 = skip the serving leg)")
    ap.add_argument("--no-schedule-comparison", action="store_true",
                    help="skip the (untimed) persistent-vs-plain schedule comparison")
    ap.add_argument("--no-graph-comparison", action="store_true",
                    help="skip the (untimed) eager-vs-graph-replay comparison")
    ap.add_argument("--autotune-cache", default="",
                    help="file of autotuner choices: written after the autotune pass, "
                         "read instead of tuning with --no-autotune")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="after the timed steps, run one plain fp64 copy kernel (y = -x) over "
                         "this many MiB, the reference dispatch for scaling HBM counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                                   "use --gpus 1 (multi-GPU sharding is a design note)"}))
        sys.exit(2)

    import torch
    from paper_1810_04758_amd import api, datagen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    api.load()
    desc, plan = WORKLOADS[args.workload]

    # synthetic inputs, generated once and made resident in HBM
    host = {}
    dev = {}
    for name, _ in plan:
        D, _, _ = datagen.config_points(name)
        host[name] = D
        dev[name] = torch.from_numpy(D).cuda()
    outs = {}
    for name, Ks in plan:
        N = host[name].shape[0]
        for K in Ks:
            outs[(name, K)] = (torch.empty((N, K), dtype=torch.int32, device="cuda"),
                               torch.empty((N, K), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    jopts = dict(lanes_per_query=args.lanes, w_factor=args.w_factor, schedule=args.schedule)

    def one_step(record):
        for name, Ks in plan:
            idx = api.build_index(dev[name], stream=stream)
            for K in Ks:
                ids, dists = outs[(name, K)]
                _, _, st = idx.self_join(K, ids=ids, dists=dists, stream=stream, with_stats=True,
                                         **jopts)
                if record is not None:
                    record.append((name, K, st))
            idx.close()

    # autotuner (untimed, like a warmup): measures the level-0 cell side and
    # the growth of the cell side per (dims, K, N) class and caches the best
    tuned = []
    if not args.no_autotune and not (args.lanes or args.w_factor):
        for name, Ks in plan:
            idx = api.build_index(dev[name], stream=stream)
            for K in Ks:
                r = idx.autotune(K, stream=stream)
                tuned.append(dict(dataset=name, K=K, w_factor=round(r["w_factor"], 3),
                                  growth=round(r["growth"], 4),
                                  linear_levels=int(r["linear_levels"]), trials=int(r["trials"]),
                                  tail_pairs=r["tail_pairs"], lanes_shift=int(r["lanes_shift"]),
                                  ms_default=round(r["ms_default"], 3),
                                  ms_tuned=round(r["ms_best"], 3)))
            idx.close()
    if args.autotune_cache:
        if tuned:
            api.autotune_save(args.autotune_cache)
        elif args.no_autotune:
            api.autotune_load(args.autotune_cache)
    for _ in range(args.warmup):
        one_step(None)
    torch.cuda.synchronize()

    records = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(records)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1000.0 / args.steps
    calib = None
    if args.calibration_copy_mib > 0:
        x = torch.ones(args.calibration_copy_mib << 17, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        calib = {"kernel": "neg (fp64 copy)", "read_bytes": x.numel() * 8,
                 "write_bytes": y.numel() * 8}
        del x, y

    queries_per_step = sum(host[name].shape[0] * len(Ks) for name, Ks in plan)
    value = queries_per_step * args.steps / elapsed

    # roofline of the search kernel (dominant kernel), from HIP events recorded
    # around its launches on the join stream
    search_ms = 0.0
    search_launches = 0
    bytes_total = 0
    ops_total = 0.0
    per_case = {}
    for name, K, st in records:
        n = host[name].shape[1]
        search_ms += sum(st["ms_search"])
        search_launches += st["levels"]
        bytes_total += alg_bytes(st, n, K)
        ops_total += alg_ops(st, n)
        c = per_case.setdefault((name, K), dict(dataset=name, K=K, ms_total=[], levels=[],
                                                fail_fraction=[], ms_search=[], ms_build=[],
                                                ms_heavy=[], ms_tail=[]))
        c["ms_heavy"].append(sum(st["ms_heavy"]))
        c["ms_tail"].append(st["ms_tail"])
        c["ms_total"].append(st["ms_total"])
        c["levels"].append(st["levels"])
        c["fail_fraction"].append(st["total_failed"] / max(1, st["total_attempted"]))
        c["ms_search"].append(sum(st["ms_search"]))
        c["ms_build"].append(sum(st["ms_build"]))
    achieved = bytes_total / (search_ms * 1e-3) / 1e9 if search_ms > 0 else 0.0
    achieved_ops = ops_total / (search_ms * 1e-3) / 1e12 if search_ms > 0 else 0.0
    # the binding roof is the one with the larger time at peak
    alu_bound = ops_total / (ALU_PEAK_TOPS * 1e12) > bytes_total / (HBM_PEAK_GBS * 1e9)
    hbm_roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    alu_roof = {"bound": "alu", "achieved": round(achieved_ops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                "unit": "TFLOP/s", "frac": round(achieved_ops / ALU_PEAK_TOPS, 4)}
    roof = dict(alu_roof if alu_bound else hbm_roof)
    roof.update({"traffic": measured_traffic(args.workload), "kernel": "k_search",
                 "alg_bytes_per_launch": round(bytes_total / max(1, search_launches)),
                 "alg_fp64_ops_per_launch": round(ops_total / max(1, search_launches)),
                 "avg_launch_ms": round(search_ms / max(1, search_launches), 4),
                 "launches": search_launches,
                 "other_roof": hbm_roof if alu_bound else alu_roof})
    cases = []
    for (name, K), c in per_case.items():
        N = host[name].shape[0]
        med = float(np.median(c["ms_total"]))
        cases.append(dict(dataset=name, K=K, N=N, ms_join_median=round(med, 3),
                          queries_per_s=round(N / (med * 1e-3), 1),
                          levels=int(np.median(c["levels"])),
                          fail_fraction=round(float(np.median(c["fail_fraction"])), 4),
                          ms_search=round(float(np.median(c["ms_search"])), 3),
                          ms_heavy=round(float(np.median(c["ms_heavy"])), 3),
                          ms_tail=round(float(np.median(c["ms_tail"])), 3),
                          ms_level_builds=round(float(np.median(c["ms_build"])), 3)))

    out = {
        "metric": "KNN self-join queries/s (1 GPU)",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": desc,
                   "queries_per_step": queries_per_step},
        "roofline": roof,
        "cases": cases,
        "autotune": tuned,
    }
    if calib:
        out["calibration_copy"] = calib
    if args.schedule == 0 and not args.no_schedule_comparison:
        out["persistent_vs_plain"] = schedule_comparison(api, dev, plan, outs, stream)
    if not args.no_graph_comparison:
        out["graph_vs_eager"] = graph_comparison(api, dev, plan, outs, stream)
    if args.serving_seconds > 0:
        out["serving"] = serving_leg(api, args.serving_seconds)
    if not args.no_cpu_baseline:
        flat = [(name, K) for name, Ks in plan for K in Ks]
        out["cpu_baseline"] = cpu_baseline(host, flat)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
