"""Benchmark of the grid KNN self-join on one MI355X.

A step is one pass of the whole hot path over the workload: for every dataset
of the workload, knn_build_index_device (bounds, eps sampling) and, for every
K, knn_self_join_device (grid levels, density-ordered persistent search,
failure re-queue and re-index), with the coordinates already resident in
device memory.  The default workload is the largest configuration, the
clustered catalogue-shaped 2-D set (N = 2e7, K = 16).  The other
configurations are reported beside it as extra cases (join time, queries/s
and the search kernel's roofline each), with the persistent-vs-plain and
graph-vs-eager comparisons, the serving workload at two request rates, and
the CPU oracle timed on every configuration.  Prints one JSON line.

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
    "clustered2d_20m": ("clustered catalogue-shaped 2-D: 70% from 500 Gaussian clusters, 30% "
                        "uniform background, N=2e7, K=16", [("clustered2d_20m", [16])]),
    "expo_2m": ("skewed density: exponential(rate 40) coordinates, N=2e6, 2-D and 4-D, "
                "K in {1,8,32,64}", [("expo2d_2m", [1, 8, 32, 64]), ("expo4d_2m", [1, 8, 32, 64])]),
    "expo2d_2m_k32": ("exponential(rate 40) 2-D, N=2e6, K=32", [("expo2d_2m", [32])]),
    "unif2d_50k": ("uniform [0,100)^2, N=5e4, K=5", [("unif2d_50k", [5])]),
    "unif6d_5m": ("uniform [0,100)^6, N=5e6, K=32", [("unif6d_5m", [32])]),
}
# the configurations reported beside the headline, as extra cases
EXTRA_WORKLOADS = ["unif2d_50k", "expo_2m", "unif6d_5m", "clustered2d_20m"]

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


def roofline_of(records):
    """Roofline of the search kernel over the given joins [(n, K, stats)]:
    algorithmic bytes and FP64 operations of all its launches over their total
    duration (HIP events recorded around each launch on the join stream).  The
    binding roof is the one with the larger time at peak; the other is
    reported beside it."""
    search_ms = sum(sum(st["ms_search"]) for _, _, st in records)
    launches = sum(st["levels"] for _, _, st in records)
    nbytes = sum(alg_bytes(st, n, K) for n, K, st in records)
    ops = sum(alg_ops(st, n) for n, K, st in records)
    achieved = nbytes / (search_ms * 1e-3) / 1e9 if search_ms > 0 else 0.0
    achieved_ops = ops / (search_ms * 1e-3) / 1e12 if search_ms > 0 else 0.0
    alu_bound = ops / (ALU_PEAK_TOPS * 1e12) > nbytes / (HBM_PEAK_GBS * 1e9)
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    alu = {"bound": "alu", "achieved": round(achieved_ops, 3), "peak": round(ALU_PEAK_TOPS, 2),
           "unit": "TFLOP/s", "frac": round(achieved_ops / ALU_PEAK_TOPS, 4)}
    roof = dict(alu if alu_bound else hbm)
    roof.update({"kernel": "k_search",
                 "alg_bytes_per_launch": round(nbytes / max(1, launches)),
                 "alg_fp64_ops_per_launch": round(ops / max(1, launches)),
                 "avg_launch_ms": round(search_ms / max(1, launches), 4),
                 "launches": launches,
                 "other_roof": hbm if alu_bound else alu})
    return roof


def oracle_rate(D, K, rows, threads):
    """Queries per second of the brute-force oracle on the given rows."""
    import oracle
    t0 = time.perf_counter()
    oracle.knn(D, K, rows=rows, threads=threads)
    return rows.shape[0] / (time.perf_counter() - t0), time.perf_counter() - t0


def cpu_baseline(cases, budget_s=3.0, single_s=1.5):
    """The CPU oracle (brute force by the definition, as it stands) timed on
    the host cores on a bounded random sample of each configuration's queries:
    all cores, then one core; a probe sizes each sample to about budget_s
    (single_s on one core) of wall time.  cases: [(name, D, K)]."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(0)
    out = []
    for name, D, K in cases:
        N = D.shape[0]
        probe = rng.choice(N, size=min(N, threads), replace=False)
        r, _ = oracle_rate(D, K, probe, threads)
        n_all = int(min(N, max(threads, min(200_000, budget_s * r))))
        rows = rng.choice(N, size=n_all, replace=False)
        r_all, t_all = oracle_rate(D, K, rows, threads)
        n_one = int(min(N, max(4, min(50_000, single_s * r_all / threads))))
        rows1 = rng.choice(N, size=n_one, replace=False)
        r_one, t_one = oracle_rate(D, K, rows1, 1)
        out.append({"config": name, "K": K, "N": N,
                    "all_cores": {"value": round(r_all, 2), "cores": threads,
                                  "sample_queries": n_all, "wall_s": round(t_all, 2)},
                    "single_core": {"value": round(r_one, 2), "cores": 1,
                                    "sample_queries": n_one, "wall_s": round(t_one, 2)}})
    return out


def serving_leg(api, seconds, rate, pool=None, idxs=None, budget_gib=96, inflight=4,
                max_queue=64):
    """The serving workload: a Poisson stream (mean `rate` requests/s for
    `seconds`) of self-join requests over 24 resident datasets (N log-uniform
    in [1e4, 1e7], dims in {2,3,4,6}, uniform or exponential coordinates, K in
    {1,4,16,64}), admitted by device-memory footprint and run concurrently.  A
    request that finds max_queue requests already waiting is refused
    (KNN_EBUSY) and counted.  Latency is submit -> results ready; most
    requests are latency-only (results discarded on the device), every 25th is
    copied back and compared with a solo join of the same index and K."""
    from paper_1810_04758_amd._lib import KNN_EBUSY, KnnError
    from paper_1810_04758_amd import datagen
    arrivals, ds, ks = datagen.serving_trace(seconds, rate, len(pool))
    srv = api.Server(mem_budget_bytes=budget_gib << 30, max_inflight=inflight,
                     max_queue=max_queue)
    for ix in idxs:
        srv.add_dataset(ix)
    checks = []
    tickets = []
    refused = 0
    t0 = time.perf_counter()
    for i, (ta, d, k) in enumerate(zip(arrivals, ds, ks)):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        N = pool[d][0].shape[0]
        keep = (i % 25 == 0) and N <= 1_000_000
        try:
            tickets.append((srv.submit(int(d), int(k), N, discard=not keep), int(d), int(k),
                            keep))
        except KnnError as e:
            if e.code != KNN_EBUSY:
                raise
            refused += 1
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
    return {"offered": int(len(arrivals)), "refused_queue_full": refused,
            "completed": int(st["completed"]), "trace_seconds": seconds, "rate_per_s": rate,
            "p50_ms": round(st["p50_ms"], 2), "p99_ms": round(st["p99_ms"], 2),
            "mean_ms": round(st["mean_ms"], 2), "queries_per_s": round(st["queries_per_s"], 1),
            "requests_per_s": round(st["requests_per_s"], 2), "wall_s": round(wall, 2),
            "peak_inflight": int(st["peak_inflight"]), "peak_bytes": int(st["peak_bytes"]),
            "max_queue": max_queue,
            "mix_equals_solo_checked": len(checks), "mix_equals_solo": same}


def serving(api, seconds_hi, seconds_lo, rate_lo):
    """Both serving points over one resident pool: the configured 200
    requests/s, and a rate the GPU sustains (served about equal to offered)."""
    from paper_1810_04758_amd import datagen
    t_build = time.perf_counter()
    pool = datagen.serving_pool()
    idxs = [api.build_index(D) for D, _ in pool]
    t_build = time.perf_counter() - t_build
    out = {"datasets": [desc for _, desc in pool], "index_build_s": round(t_build, 2)}
    if seconds_lo > 0:
        out["sustainable"] = serving_leg(api, seconds_lo, rate_lo, pool, idxs)
    if seconds_hi > 0:
        out["configured"] = serving_leg(api, seconds_hi, 200.0, pool, idxs)
    for ix in idxs:
        ix.close()
    return out


def schedule_row(idx, K, ids, dists, stream, reps=3):
    """The persistent schedule (device work queues per XCD, density-ordered
    items, heavy queries on workgroups of their own) against the plain one:
    one launch per level over every unsolved query in cell order, one work
    item per wavefront, no queue (same cell sides and lanes per query, so the
    same candidates are scanned).  Best of `reps` joins each; search time
    (both search kernels) from the join's HIP events."""
    row = {}
    for sched in (0, 1):
        best_s = best_t = float("inf")
        extra = dict(schedule=1, heavy_min=-1) if sched else {}
        for _ in range(reps):
            _, _, st = idx.self_join(K, ids=ids, dists=dists, stream=stream, with_stats=True,
                                     **extra)
            best_s = min(best_s, sum(st["ms_search"]) + sum(st["ms_heavy"]))
            best_t = min(best_t, st["ms_total"])
        key = "persistent" if sched == 0 else "plain"
        row[f"ms_search_{key}"] = round(best_s, 3)
        row[f"ms_join_{key}"] = round(best_t, 3)
    row["search_speedup"] = round(row["ms_search_plain"] / row["ms_search_persistent"], 3)
    row["join_speedup"] = round(row["ms_join_plain"] / row["ms_join_persistent"], 3)
    return row


def graph_row(idx, K, ids, dists, stream, reps=3):
    """Eager joins against replays of the join captured in a HIP graph
    (use_graph): same index, K and outputs; wall time from submit to the
    stream being drained, best of `reps` each."""
    import torch
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
    return dict(ms_eager=round(best[0], 3), ms_graph_replay=round(best[1], 3),
                speedup=round(best[0] / best[1], 3))


def tune_row(r):
    return dict(w_factor=round(r["w_factor"], 4), growth=round(r["growth"], 4),
                linear_levels=int(r["linear_levels"]), zorder=int(r["zorder"]),
                trials=int(r["trials"]), tail_pairs=r["tail_pairs"],
                lanes_shift=int(r["lanes_shift"]), queue_pops=int(r["queue_pops"]),
                ms_default=round(r["ms_default"], 3),
                ms_tuned=round(r["ms_best"], 3))


def case_summary(name, K, N, sts):
    """Medians over the timed joins of one (dataset, K)."""
    med = lambda key: float(np.median([key(st) for st in sts]))  # noqa: E731
    ms = med(lambda st: st["ms_total"])
    return dict(dataset=name, K=K, N=N, ms_join_median=round(ms, 3),
                queries_per_s=round(N / (ms * 1e-3), 1),
                levels=int(med(lambda st: st["levels"])),
                fail_fraction=round(med(lambda st: st["total_failed"] /
                                        max(1, st["total_attempted"])), 4),
                ms_search=round(med(lambda st: sum(st["ms_search"])), 3),
                ms_heavy=round(med(lambda st: sum(st["ms_heavy"])), 3),
                ms_tail=round(med(lambda st: st["ms_tail"]), 3),
                ms_level_builds=round(med(lambda st: sum(st["ms_build"])), 3))


def extra_cases(api, stream, names, autotune, reps, sched_sets, graph_sets, host_keep):
    """The other configurations: per (dataset, K) an untimed autotune pass and
    a warm-up join, then `reps` timed joins (index built once, inputs and
    outputs resident); the join median, queries/s and the search kernel's
    roofline per configuration; persistent-vs-plain on sched_sets and
    graph-vs-eager on graph_sets."""
    import torch
    from paper_1810_04758_amd import datagen
    out, sched, graph = [], [], []
    for wl in names:
        desc, plan = WORKLOADS[wl]
        recs = []
        cases = []
        for name, Ks in plan:
            D, _, _ = datagen.config_points(name)
            host_keep[name] = D
            Dd = torch.from_numpy(D).cuda()
            N, n = D.shape
            idx = api.build_index(Dd, stream=stream)
            for K in Ks:
                ids = torch.empty((N, K), dtype=torch.int32, device="cuda")
                dists = torch.empty((N, K), dtype=torch.float64, device="cuda")
                tuned = tune_row(idx.autotune(K, stream=stream)) if autotune else None
                idx.self_join(K, ids=ids, dists=dists, stream=stream)
                sts = []
                for _ in range(reps):
                    _, _, st = idx.self_join(K, ids=ids, dists=dists, stream=stream,
                                             with_stats=True)
                    sts.append(st)
                    recs.append((n, K, st))
                c = case_summary(name, K, N, sts)
                c["roofline"] = roofline_of([(n, K, st) for st in sts])
                if tuned:
                    c["autotune"] = tuned
                cases.append(c)
                if wl in sched_sets:
                    sched.append(dict(dataset=name, K=K, **schedule_row(idx, K, ids, dists,
                                                                        stream)))
                if wl in graph_sets:
                    graph.append(dict(dataset=name, K=K, **graph_row(idx, K, ids, dists, stream)))
                del ids, dists
            idx.close()
            del Dd
            torch.cuda.empty_cache()
        out.append(dict(workload=wl, description=desc, cases=cases, roofline=roofline_of(recs)))
    return out, sched, graph


def _eps_for(idx, per_point, lo, hi, stride=64):
    """eps holding about per_point pairs per point, by bisection on the
    sampled result-size estimate (knn_eps_join_size with a stride)."""
    for _ in range(40):
        mid = (lo * hi) ** 0.5
        if idx.eps_join_size(mid, sample_stride=stride) > per_point * idx.N:
            hi = mid
        else:
            lo = mid
        if hi / lo < 1.02:
            break
    return hi


def eps_join_leg(api, huge=True):
    """The distance similarity self-join (every pair within eps) on three
    workloads, eps chosen for a fixed mean pair count per point: level and
    exact counts, the device write of all pairs as one batch (the write
    kernel's output rate against HBM), the sampled estimate's error, and the
    host streaming rate on 3 streams.  With `huge`, the clustered set at the
    KNN method's eps_min(16): a result far larger than HBM streamed to host."""
    import torch
    from paper_1810_04758_amd import datagen
    rows = []
    dev = torch.device("cuda", 0)
    for name, per_point, lo, hi in [("expo2d_2m", 32, 1e-6, 1.0), ("unif6d_5m", 32, 0.1, 100.0),
                                    ("clustered2d_20m", 16, 1e-5, 10.0)]:
        D, _, _ = datagen.config_points(name)
        Dd = torch.from_numpy(D).cuda()
        idx = api.build_index(Dd)
        eps = _eps_for(idx, per_point, lo, hi)
        idx.eps_join_release()  # time the level build and the counts from scratch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total = idx.eps_join_size(eps)
        ms_count = 1e3 * (time.perf_counter() - t0)
        est = idx.eps_join_size(eps, sample_stride=64)
        idx.eps_join_size(eps)  # exact counts again for the batches
        q = torch.empty(total, dtype=torch.int32, device=dev)
        j = torch.empty(total, dtype=torch.int32, device=dev)
        d = torch.empty(total, dtype=torch.float64, device=dev)
        best = None
        for _ in range(3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            n, nxt = idx.eps_join_batch(eps, 0, q, j, d)
            b.record()
            torch.cuda.synchronize()
            assert n == total and nxt == idx.N
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        del q, j, d
        torch.cuda.empty_cache()
        st = idx.eps_join(eps, consume=lambda *_: False, batch_pairs=1 << 24, n_streams=3)
        body = st["ms_total"] - st["ms_count"]
        out_gb = total * 16 / 1e9
        rows.append({
            "dataset": name, "N": int(D.shape[0]), "eps": eps, "pairs": int(total),
            "pairs_per_point": round(total / D.shape[0], 2),
            "ms_level_and_counts": round(ms_count, 3),
            "estimate_stride64_rel_err": round(est / total - 1.0, 5),
            "ms_write_device": round(best, 3),
            "pairs_per_s_device": round(total / (best / 1e3), 1),
            "write_roofline": {"bound": "hbm", "achieved": round(out_gb / (best / 1e3), 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(out_gb / (best / 1e3) / HBM_PEAK_GBS, 4),
                               "bytes": "16 B of output per pair (the written result only)"},
            "host_stream_3x2^24": {"ms": round(body, 2), "GB_per_s": round(out_gb / (body / 1e3), 2),
                                   "batches": st["n_batches"]}})
        print(f"[bench] eps join {name}: {rows[-1]['pairs']} pairs, write "
              f"{rows[-1]['ms_write_device']} ms", file=sys.stderr, flush=True)
        if huge and name == "clustered2d_20m":
            eh = idx.eps_min(16)
            seen = [0]

            def cons(qa, ja, da):
                seen[0] += qa.size
                return False
            st = idx.eps_join(eh, consume=cons, batch_pairs=1 << 26, n_streams=3)
            body = st["ms_total"] - st["ms_count"]
            gb = st["n_pairs"] * 16 / 1e9
            rows.append({"dataset": name, "N": int(D.shape[0]), "eps": eh,
                         "eps_is": "eps_min(16) of the KNN method",
                         "pairs": int(st["n_pairs"]), "result_GB": round(gb, 1),
                         "hbm_GB": round(torch.cuda.get_device_properties(0).total_memory / 1e9, 1),
                         "host_stream_3x2^26": {"ms_total": round(st["ms_total"], 1),
                                                "ms_count": round(st["ms_count"], 1),
                                                "GB_per_s": round(gb / (body / 1e3), 2),
                                                "batches": st["n_batches"],
                                                "pairs_consumed": int(seen[0])}})
            print(f"[bench] eps join beyond HBM: {gb:.1f} GB in {st['ms_total']:.0f} ms",
                  file=sys.stderr, flush=True)
        idx.close()
        del Dd
        torch.cuda.empty_cache()
    return rows


def hybrid_leg(api):
    """The hybrid CPU/GPU join (host outputs) beside the GPU-only join with
    host outputs (knn_self_join) on the same workload: times, the split and
    the load imbalance |T_CPU - T_GPU| / T; the hybrid's second call (its
    kd-tree is built by the first and kept with the index)."""
    import torch
    from paper_1810_04758_amd import datagen
    rows = []
    for name, K in [("expo2d_2m", 32), ("clustered2d_20m", 16)]:
        D, _, _ = datagen.config_points(name)
        idx = api.build_index(torch.from_numpy(D).cuda())
        gi, gd = idx.self_join_host(K)
        t0 = time.perf_counter()
        gi, gd = idx.self_join_host(K)
        ms_gpu_only = 1e3 * (time.perf_counter() - t0)
        _, _, st0 = idx.self_join_hybrid(K)
        hi, hd, st = idx.self_join_hybrid(K)
        same = bool(np.array_equal(hi, gi) and np.array_equal(hd, gd))
        rows.append({"dataset": name, "K": K, "ms_gpu_only_host_out": round(ms_gpu_only, 2),
                     "ms_hybrid": round(st["ms_total"], 2),
                     "ms_T_gpu": round(st["ms_gpu"], 2), "ms_T_cpu": round(st["ms_cpu"], 2),
                     "load_imbalance": round(st["load_imbalance"], 4),
                     "ms_queue": round(st["ms_queue"], 2), "ms_merge": round(st["ms_merge"], 2),
                     "ms_cpu_index_first_call": round(st0["ms_cpu_index"], 1),
                     "gpu_queries": st["gpu_queries"], "cpu_queries": st["cpu_queries"],
                     "gpu_batches": st["gpu_batches"],
                     "monolithic_batches": st["monolithic_batches"],
                     "reindexes": st["reindexes"], "cpu_threads": st["cpu_threads"],
                     "same_rows_as_gpu_only": same})
        print(f"[bench] hybrid {name}: {rows[-1]['ms_hybrid']} ms vs GPU-only "
              f"{rows[-1]['ms_gpu_only_host_out']} ms", file=sys.stderr, flush=True)
        idx.close()
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clustered2d_20m", choices=sorted(WORKLOADS))
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--w-factor", type=float, default=0.0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the (untimed) knn_autotune pass before the timed steps")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other configurations (extra cases)")
    ap.add_argument("--extra-reps", type=int, default=5,
                    help="timed joins per extra case")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the 200 requests/s serving trace (0 = skip)")
    ap.add_argument("--serving-sustainable-seconds", type=float, default=20.0,
                    help="length of the serving trace at the sustainable rate (0 = skip)")
    ap.add_argument("--serving-sustainable-rate", type=float, default=10.0,
                    help="requests/s of the sustainable serving point")
    ap.add_argument("--no-schedule-comparison", action="store_true",
                    help="skip the (untimed) persistent-vs-plain schedule comparison")
    ap.add_argument("--no-graph-comparison", action="store_true",
                    help="skip the (untimed) eager-vs-graph-replay comparison")
    ap.add_argument("--autotune-cache", default="",
                    help="file of autotuner choices: written after the autotune pass, "
                         "read instead of tuning with --no-autotune")
    ap.add_argument("--no-eps-join", action="store_true",
                    help="skip the distance similarity self-join leg")
    ap.add_argument("--no-eps-huge", action="store_true",
                    help="skip the eps join whose result is larger than HBM (streamed to host)")
    ap.add_argument("--no-hybrid", action="store_true",
                    help="skip the hybrid CPU/GPU join leg")
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
    print(f"[bench] workload {args.workload}", file=sys.stderr, flush=True)

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

    # autotuner (untimed, like a warmup): measures the level-0 cell side, the
    # level structure and the growth of the cell side per (dims, K, N) class
    # and caches the best
    tuned = []
    if not args.no_autotune and not (args.lanes or args.w_factor):
        for name, Ks in plan:
            idx = api.build_index(dev[name], stream=stream)
            for K in Ks:
                tuned.append(dict(dataset=name, K=K, **tune_row(idx.autotune(K, stream=stream))))
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
    print(f"[bench] timed steps done: {ms_per_step:.3f} ms per step", file=sys.stderr, flush=True)
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
    roof = roofline_of([(host[name].shape[1], K, st) for name, K, st in records])
    roof["traffic"] = measured_traffic(args.workload)
    per_case = {}
    for name, K, st in records:
        per_case.setdefault((name, K), []).append(st)
    cases = [case_summary(name, K, host[name].shape[0], sts) for (name, K), sts in
             per_case.items()]

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
    cmp_sched = args.schedule == 0 and not args.no_schedule_comparison
    cmp_graph = not args.no_graph_comparison
    sched_rows, graph_rows = [], []
    if cmp_sched or cmp_graph:
        for name, Ks in plan:
            idx = api.build_index(dev[name], stream=stream)
            for K in Ks:
                ids, dists = outs[(name, K)]
                if cmp_sched:
                    sched_rows.append(dict(dataset=name, K=K,
                                           **schedule_row(idx, K, ids, dists, stream)))
                if cmp_graph and args.workload in ("clustered2d_20m", "unif6d_5m"):
                    graph_rows.append(dict(dataset=name, K=K,
                                           **graph_row(idx, K, ids, dists, stream)))
            idx.close()
    # the headline's device buffers are not needed past this point
    del outs
    dev.clear()
    torch.cuda.empty_cache()
    if not args.no_extra:
        names = [w for w in EXTRA_WORKLOADS if w != args.workload]
        print(f"[bench] extra cases {names}", file=sys.stderr, flush=True)
        extra, s2, g2 = extra_cases(
            api, stream, names, not args.no_autotune, args.extra_reps,
            sched_sets={"expo_2m", "clustered2d_20m"} if cmp_sched else set(),
            graph_sets={"unif6d_5m", "clustered2d_20m"} if cmp_graph else set(),
            host_keep=host)
        out["extra_cases"] = extra
        sched_rows += s2
        graph_rows += g2
    if sched_rows:
        tp = sum(r["ms_search_plain"] for r in sched_rows)
        tq = sum(r["ms_search_persistent"] for r in sched_rows)
        jp = sum(r["ms_join_plain"] for r in sched_rows)
        jq = sum(r["ms_join_persistent"] for r in sched_rows)
        out["persistent_vs_plain"] = {"cases": sched_rows, "search_speedup": round(tp / tq, 3),
                                      "join_speedup": round(jp / jq, 3)}
    if graph_rows:
        te = sum(r["ms_eager"] for r in graph_rows)
        tg = sum(r["ms_graph_replay"] for r in graph_rows)
        out["graph_vs_eager"] = {"cases": graph_rows, "speedup": round(te / tg, 3)}
    if not args.no_eps_join:
        print("[bench] eps join", file=sys.stderr, flush=True)
        out["eps_join"] = eps_join_leg(api, huge=not args.no_eps_huge)
    if not args.no_hybrid:
        print("[bench] hybrid", file=sys.stderr, flush=True)
        out["hybrid"] = hybrid_leg(api)
    if args.serving_seconds > 0 or args.serving_sustainable_seconds > 0:
        print("[bench] serving", file=sys.stderr, flush=True)
        out["serving"] = serving(api, args.serving_seconds, args.serving_sustainable_seconds,
                                 args.serving_sustainable_rate)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cfgs = [(name, host[name], K) for name, Ks in plan for K in Ks]
        for wl in (EXTRA_WORKLOADS if not args.no_extra else []):
            if wl == args.workload:
                continue
            for name, Ks in WORKLOADS[wl][1]:
                cfgs += [(name, host[name], K) for K in Ks[:1]]
        per = cpu_baseline(cfgs)
        head = per[0]["all_cores"]
        out["cpu_baseline"] = {
            "value": head["value"], "unit": "queries/s", "cores": head["cores"],
            "kind": "oracle",
            "sample": (f"brute-force oracle (the definition, OpenMP over queries) on "
                       f"{head['sample_queries']} random rows of {per[0]['config']} at "
                       f"K={per[0]['K']} ({head['wall_s']} s wall); single core: "
                       f"{per[0]['single_core']['value']} queries/s on "
                       f"{per[0]['single_core']['sample_queries']} rows"),
            "per_config": per}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
