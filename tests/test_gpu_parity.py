"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Neighbour ids must be identical and distances bit-identical (0 ulp): both
sides sum the squared distance left to right with every operation rounded
and take a correctly rounded square root.
"""

import json
import os
import sys

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def knn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04758_amd import api
    api.load()
    return api


def _check_rows(D, ids, dists, K, rows, oracle_mod):
    ref_ids, ref_d = oracle_mod.knn(D, K, rows=rows)
    got_ids = ids[rows]
    got_d = dists[rows]
    bad = np.nonzero((got_ids != ref_ids).any(axis=1) | (got_d != ref_d).any(axis=1))[0]
    assert bad.size == 0, (f"{bad.size} rows differ; first row {rows[bad[0]]}: "
                           f"got {got_ids[bad[0]].tolist()} {got_d[bad[0]].tolist()} "
                           f"want {ref_ids[bad[0]].tolist()} {ref_d[bad[0]].tolist()}")


def _join(knn, D, K, device_input=True, **opts):
    import torch
    if device_input:
        idx = knn.build_index(torch.from_numpy(D).cuda())
    else:
        idx = knn.build_index(D)
    ids, dists, st = idx.self_join(K, with_stats=True, **opts)
    torch.cuda.synchronize()
    out = ids.cpu().numpy(), dists.cpu().numpy(), st
    idx.close()
    return out


CASES = [
    # (name, generator, N, n, K)
    ("unif2d", lambda: datagen.uniform(3001, 2, seed=21), 3001, 2, 5),
    ("unif3d", lambda: datagen.uniform(2999, 3, seed=22), 2999, 3, 8),
    ("expo4d", lambda: datagen.exponential(4099, 4, seed=23), 4099, 4, 16),
    ("unif5d", lambda: datagen.uniform(2050, 5, seed=24), 2050, 5, 3),
    ("unif6d", lambda: datagen.uniform(3000, 6, seed=25), 3000, 6, 32),
    ("clus2d", lambda: datagen.clustered(5003, seed=26), 5003, 2, 16),
    ("expo2d_k64", lambda: datagen.exponential(4001, 2, seed=27), 4001, 2, 64),
    ("expo2d_k1", lambda: datagen.exponential(4001, 2, seed=28), 4001, 2, 1),
]


@pytest.mark.parametrize("name,gen,N,n,K", CASES, ids=[c[0] for c in CASES])
def test_parity_full(knn, oracle_mod, name, gen, N, n, K):
    D = gen()
    _say(f"[parity_full] {name} N={N} n={n} K={K}")
    ids, dists, st = _join(knn, D, K)
    _check_rows(D, ids, dists, K, np.arange(N), oracle_mod)
    assert st["total_failed"] <= st["total_attempted"]


def test_parity_host_entry_point(knn, oracle_mod):
    D = datagen.exponential(2500, 3, seed=31)
    _say("[parity_host] knn_build_index + knn_self_join N=2500 n=3 K=7")
    idx = knn.build_index(D)
    ids, dists = idx.self_join_host(7)
    idx.close()
    _check_rows(D, ids, dists, 7, np.arange(2500), oracle_mod)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
def test_lanes_per_query(knn, oracle_mod, lanes):
    D = datagen.exponential(3333, 2, seed=32)
    _say(f"[lanes] T={lanes}")
    ids, dists, _ = _join(knn, D, 12, lanes_per_query=lanes)
    _check_rows(D, ids, dists, 12, np.arange(3333), oracle_mod)


@pytest.mark.parametrize("wf", [0.25, 0.5, 1.0, 2.0, 4.0])
@pytest.mark.parametrize("schedule", [0, 1])
def test_w_factor_and_schedule_metamorphic(knn, oracle_mod, wf, schedule):
    # the result may not depend on the cell side or the schedule (Sec. 5,
    # sensitivity to the initial eps, factors 0.25x..4x)
    D = datagen.uniform(2777, 4, seed=33)
    _say(f"[w_factor] wf={wf} schedule={schedule}")
    ids, dists, st = _join(knn, D, 9, w_factor=wf, schedule=schedule, batch_queries=640)
    _check_rows(D, ids, dists, 9, np.arange(2777), oracle_mod)
    if wf <= 0.25:
        assert st["total_failed"] > 0  # forced failures ran
    # same with the brute-force tail off: failures go through re-indexing only
    ids2, dists2, st2 = _join(knn, D, 9, w_factor=wf, schedule=schedule, tail_pairs=-1.0)
    assert (ids2 == ids).all() and (dists2 == dists).all()
    if wf <= 0.25:
        assert st2["levels"] > 1 and st2["tail_queries"] == 0


@pytest.mark.parametrize("tail", [-1.0, 1e15, 0.0])
def test_tail_modes(knn, oracle_mod, tail):
    # brute-force tail disabled / for every failure of level 0 / default budget:
    # identical results (skewed data with duplicates, K large enough that the
    # tail's per-query buffers need the exact bisection on ties)
    base = datagen.exponential(2400, 2, seed=34)
    D = np.concatenate([base, base[:300], base[:300]])
    _say(f"[tail] tail_pairs={tail}")
    ids, dists, st = _join(knn, D, 24, tail_pairs=tail, w_factor=0.5)
    _check_rows(D, ids, dists, 24, np.arange(D.shape[0]), oracle_mod)
    if tail == 1e15:
        assert st["tail_queries"] > 0 and st["levels"] == 1
    if tail < 0:
        assert st["tail_queries"] == 0


def test_tail_all_duplicates(knn, oracle_mod):
    # every query in the tail sees all N-1 points at distance 0: the selection
    # must fall back on ids (exact bisection over the id bits)
    D = np.full((700, 4), 3.5)
    D[:10] = datagen.uniform(10, 4, seed=35)
    _say("[tail] all duplicates")
    ids, dists, st = _join(knn, D, 40, tail_pairs=1e15, w_factor=0.25)
    _check_rows(D, ids, dists, 40, np.arange(D.shape[0]), oracle_mod)


def test_figures_through_gpu(knn, oracle_mod):
    for name in ("fig_eps_expansion.json", "fig_work_example.json"):
        g = json.load(open(os.path.join(GOLDEN, name)))
        panels = g["panels"].values() if "panels" in g else [g]
        for p in panels:
            D = np.array(p["points"], dtype=np.float64)
            K = D.shape[0] - 1
            _say(f"[figure] {name} N={D.shape[0]} K={K}")
            ids, dists, _ = _join(knn, D, K)
            _check_rows(D, ids, dists, K, np.arange(D.shape[0]), oracle_mod)
            kk = len(p["knn_ids_of_query"])
            assert ids[0, :kk].tolist() == p["knn_ids_of_query"]


@pytest.mark.parametrize("case", ["dups", "all_same", "n2", "lattice", "kmax", "line",
                                  "outliers3d", "outliers4d", "outliers2d"])
def test_edge_cases(knn, oracle_mod, case):
    if case == "dups":
        base = datagen.uniform(300, 2, seed=40)
        D = np.concatenate([base] * 7)  # every point 7 times
        K = 10
    elif case == "all_same":
        D = np.full((500, 3), 1.25)
        K = 17
    elif case == "n2":
        D = np.array([[0.0, 0.0], [1.0, 2.0]])
        K = 1
    elif case == "lattice":
        D = datagen.lattice(12, 2)
        K = 12
    elif case == "kmax":
        D = datagen.uniform(300, 2, seed=41)
        K = 299
    elif case.startswith("outliers"):
        # a small dense cube and a few points 1e4 away: the grid has far more
        # rows than points (and cells than the key space allows at first), so
        # neighbour ranges come from binary search over the cell keys rather
        # than a dense or row table
        n = int(case[-2])
        D = datagen.uniform(3000, n, seed=44) / 100.0
        D = np.concatenate([D, np.full((3, n), 1e4) + np.arange(3)[:, None]])
        K = 5
    else:  # all points on a line (zero extent in one dimension)
        D = np.zeros((1000, 2))
        D[:, 0] = np.linspace(0, 1, 1000) ** 2
        K = 6
    _say(f"[edge] {case} N={D.shape[0]} K={K}")
    ids, dists, _ = _join(knn, D, K)
    _check_rows(D, ids, dists, K, np.arange(D.shape[0]), oracle_mod)


def test_autotune_keeps_results_and_roundtrips(knn, oracle_mod, tmp_path):
    import torch
    D = datagen.exponential(6000, 3, seed=36)
    _say("[autotune]")
    idx = knn.build_index(torch.from_numpy(D).cuda())
    r = idx.autotune(10)
    # 17-20 row-major trials, 10 Z-order ones (2-4 dimensions), 2 more when
    # Z-order levels win, one without the linear step, 2 lanes shifts, 4
    # queue granularities and 2 final sides
    assert 32 <= r["trials"] <= 40 and r["ms_best"] <= r["ms_default"] and r["tail_pairs"] > 0
    assert r["queue_pops"] in (4, 8, 16, 32, 64)
    assert r["lanes_shift"] in (-1, 0, 1) and r["zorder"] in (-1, 1)
    assert r["w_factor"] > 0 and r["growth"] > 1 and r["linear_levels"] in (1, -1)
    ids, dists = idx.self_join(10)  # uses the cached setting
    torch.cuda.synchronize()
    idx.close()
    _check_rows(D, ids.cpu().numpy(), dists.cpu().numpy(), 10, np.arange(6000), oracle_mod)
    path = str(tmp_path / "tune.txt")
    knn.autotune_save(path)
    line = open(path).read().split()
    assert len(line) % 11 == 0 and len(line) >= 11
    knn.autotune_load(path)


def test_invalid_arguments(knn):
    import torch
    from paper_1810_04758_amd._lib import KnnError, KNN_EINVAL
    with pytest.raises(KnnError) as e:
        knn.build_index(np.zeros((10, 7)))
    assert e.value.code == KNN_EINVAL
    bad = datagen.uniform(100, 2, seed=1)
    bad[5, 1] = np.nan
    with pytest.raises(KnnError):
        knn.build_index(torch.from_numpy(bad).cuda())
    idx = knn.build_index(datagen.uniform(100, 2, seed=1))
    with pytest.raises(KnnError):
        idx.self_join(100)
    with pytest.raises(KnnError):
        idx.self_join(0)
    with pytest.raises(KnnError):
        idx.self_join(5, lanes_per_query=3)
    idx.close()


def test_grid_export_matches_oracle(knn, oracle_mod):
    for n, gen, w in ((2, lambda: datagen.exponential(5000, 2, seed=50), 0.01),
                      (4, lambda: datagen.uniform(4000, 4, seed=51), 17.0),
                      (6, lambda: datagen.uniform(3000, 6, seed=52), 30.0)):
        D = gen()
        _say(f"[grid_export] n={n} w={w}")
        idx = knn.build_index(D)
        got = idx.grid_export(w)
        idx.close()
        ref = oracle_mod.grid(D, 1.0 / w)
        assert (got["g"] == ref["g"]).all()
        assert (got["sorted_keys"] == ref["sorted_keys"]).all()
        assert (got["perm"] == ref["perm"]).all()
        assert (got["cell_keys"] == ref["cell_keys"]).all()
        assert (got["cell_start"] == ref["cell_start"]).all()
        assert (got["ranges"] == ref["ranges"]).all()


@pytest.mark.parametrize("scale", [1.0, 2.0 ** -70, 2.0 ** 70])
def test_sampling_kernels_match_oracle(knn, oracle_mod, scale):
    """The two sampling kernels of Sec. 4.4 on the same sample as the oracle;
    scaled inputs put d^2 outside float's normal range (the kernel's
    single-precision bin estimate must then give way to fp64)."""
    import torch
    D = datagen.exponential(20000, 3, seed=60) * scale
    sample = datagen.sample_ids(20000, 300, seed=61)
    Dd = torch.from_numpy(D).cuda()
    sd = torch.from_numpy(sample).cuda()
    _say(f"[sampling] mean + histogram scale={scale}")
    m = knn.sample_mean_dist(Dd, sd)
    m_ref = oracle_mod.sample_mean_dist(D, sample)
    # both sum the same 44850 positive terms in different orders: each sum is
    # within (terms - 1) * 2^-53 (relative) of the exact one
    assert abs(m - m_ref) <= 2 * 44850 * 2.0 ** -53 * m_ref
    inv_bw = 1000.0 / m_ref
    counts = knn.dist_histogram(Dd, sd[:50], inv_bw, 1000).cpu().numpy().astype(np.uint64)
    ref = oracle_mod.dist_histogram(D, sample[:50], inv_bw, 1000)
    assert (counts == ref).all()


@pytest.mark.parametrize("name,gen,seed", [
    ("expo2d", lambda: datagen.exponential(300_000, 2, seed=62), 1),
    ("clustered", lambda: datagen.clustered(400_000, seed=63), 77),
    ("unif4d", lambda: datagen.uniform(100_000, 4, seed=64), 5),
    ("small_fallback", lambda: datagen.uniform(1100, 2, seed=65), 9),
    # scaled far from 1: the single-precision rejection of far pairs is off
    # below (squares near float's subnormal range) and checked above
    ("unif2d_tiny", lambda: datagen.uniform(100_000, 2, seed=67) * 2.0 ** -70, 3),
    ("expo3d_large", lambda: datagen.exponential(100_000, 3, seed=68) * 2.0 ** 40, 4),
    ("clustered_offset", lambda: datagen.clustered(300_000, seed=69) + 3.0e6, 5),
    # large enough for the histogram's estimate on a point subset: bins are
    # counted only up to about where K = 1024 is reached
    ("clustered_2m", lambda: datagen.clustered(2_200_000, seed=66), 3),
])
def test_eps_min_chain_matches_oracle(knn, oracle_mod, name, gen, seed):
    """The whole Sec. 4.4 chain of an index against the oracle's own: sample
    ids (drawn on the oracle side with its own SplitMix64), eps_mean, the
    distance histogram at the oracle's bin width, and eps_min(K) by the rule
    (the midpoint of the first bin whose cumulative count reaches K per
    sample point; eps_mean when none does, as for K = 1024 on 1100 points)."""
    D = gen()
    N = D.shape[0]
    _say(f"[eps chain] {name} N={N}")
    idx = knn.build_index(D, seed=seed)
    info = idx.info()
    smp = idx.sampling()
    n_mean = min(max(int(round(0.001 * N)), 64), N, 20000)
    ref_mean_ids = oracle_mod.sample_ids(N, n_mean, seed)
    ref_hist_ids = oracle_mod.sample_ids(N, 500, seed ^ 0x5DEECE66D)
    assert (smp["mean_sample"] == ref_mean_ids).all()
    assert (smp["hist_sample"] == ref_hist_ids).all()
    eps_ref = oracle_mod.sample_mean_dist(D, ref_mean_ids)
    pairs = n_mean * (n_mean - 1) // 2
    tol = 2 * pairs * 2.0 ** -53  # two sums of `pairs` positive terms, any order
    assert abs(info["eps_mean"] - eps_ref) <= tol * eps_ref
    bw_ref = eps_ref / 1000
    counts_ref = oracle_mod.dist_histogram(D, ref_hist_ids, 1.0 / bw_ref, 1000)
    # exact up to at least the first bin where the cumulative count reaches
    # KNN_MAX_K = 1024 per sample point (all that any eps_min(K) reads), not
    # counted (0) after the first difference
    diff = np.nonzero(smp["counts"] != counts_ref)[0]
    if diff.size:
        first = diff[0]
        assert (smp["counts"][first:] == 0).all()
        assert first > 0 and np.cumsum(counts_ref)[first - 1] >= 1024 * ref_hist_ids.shape[0]
    Ks = (1, 8, 32, 64, 1024) if N > 2000 else (1, 8, 1024)
    for K in Ks:
        e_ref = oracle_mod.eps_min(counts_ref, bw_ref, ref_hist_ids.shape[0], K)
        assert abs(idx.eps_min(K) - e_ref) <= 2 * tol * e_ref, K
    if N <= 2000:
        assert idx.eps_min(1024) == info["eps_mean"] or abs(
            idx.eps_min(1024) - info["eps_mean"]) <= 4 * 2.0 ** -53 * info["eps_mean"]
    idx.close()


def test_histogram_estimate_fallback(knn, oracle_mod):
    """The index's histogram estimates, on every 8th point, the bin where the
    cumulative count reaches KNN_MAX_K = 1024 per sample point and counts
    exactly only up to it; when the exact counts then fall short, every bin
    is counted.  Built to fall short: the 500 sample points (their ids are
    known from the seed) and 520 more points, all at multiples of 8, sit in a
    unit square, the rest of the 2.1e6 points some 1000 units away.  The
    subset then sees 8 x its share of the close pairs (an estimate of about
    2.3e6 >= 4 x 512000), the exact count is about 509500 < 512000, so the
    whole histogram must come out, equal to the oracle's."""
    N = 2_100_000
    seed = 11
    hist_ids = oracle_mod.sample_ids(N, 500, seed ^ 0x5DEECE66D)
    rng = np.random.default_rng(12)
    D = rng.uniform(1000.0, 2000.0, size=(N, 2))
    near = np.setdiff1d(np.arange(0, N, 8), hist_ids)[:520]
    close = np.concatenate([hist_ids, near])
    D[close] = rng.uniform(0.0, 1.0, size=(close.shape[0], 2))
    _say(f"[histogram fallback] N={N}")
    idx = knn.build_index(D, seed=seed)
    smp = idx.sampling()
    info = idx.info()
    assert (smp["hist_sample"] == hist_ids).all()
    counts_ref = oracle_mod.dist_histogram(D, hist_ids, 1.0 / smp["bin_width"], 1000)
    c = np.cumsum(counts_ref)
    assert c[-1] < 1024 * 500 or (c >= 1024 * 500).argmax() > 2  # the estimate falls short
    assert (smp["counts"] == counts_ref).all()
    for K in (1, 64, 1024):
        e_ref = oracle_mod.eps_min(counts_ref, smp["bin_width"], 500, K)
        assert idx.eps_min(K) == e_ref, K
    assert info["n_bins"] == 1000
    idx.close()


GRAPH_CASES = [
    # (name, generator, K, options): several levels, the 5-6-D range sizing
    # and the brute-force tail all have to replay
    ("expo2d", lambda: datagen.exponential(20011, 2, seed=31), 8, {}),
    ("unif6d", lambda: datagen.uniform(6007, 6, seed=32), 8, {}),
    ("expo3d_tail", lambda: datagen.exponential(12001, 3, seed=33), 16,
     {"w_factor": 0.3, "growth": 1.3, "tail_pairs": 2e6}),
    ("expo2d_plain", lambda: datagen.exponential(9001, 2, seed=34), 4, {"schedule": 1,
                                                                        "batch_queries": 1000}),
]


@pytest.mark.parametrize("name,gen,K,opts", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_graph_replay(knn, oracle_mod, name, gen, K, opts):
    """use_graph: the capturing join and every replay give the eager result
    bit for bit, also after eager joins of another K on the same index, and
    new output buffers trigger a new capture."""
    import torch
    D = gen()
    N = D.shape[0]
    _say(f"[graph_replay] {name} N={N} K={K} {opts}")
    idx = knn.build_index(torch.from_numpy(D).cuda())
    ref_i, ref_d, st_e = idx.self_join(K, with_stats=True, **opts)
    ref_i, ref_d = ref_i.cpu().numpy(), ref_d.cpu().numpy()
    _check_rows(D, ref_i, ref_d, K, np.arange(0, N, 7), oracle_mod)
    gi = torch.empty((N, K), dtype=torch.int32, device="cuda")
    gd = torch.empty((N, K), dtype=torch.float64, device="cuda")
    for rep in range(4):
        gi.fill_(-1)
        gd.fill_(float("nan"))
        if rep == 2:  # an eager join of another K in between
            idx.self_join(K + 1)
        _, _, st = idx.self_join(K, ids=gi, dists=gd, with_stats=True, use_graph=1, **opts)
        torch.cuda.synchronize()
        assert (gi.cpu().numpy() == ref_i).all(), f"replay {rep}: ids differ"
        assert (gd.cpu().numpy() == ref_d).all(), f"replay {rep}: distances differ"
        assert st["levels"] == st_e["levels"]
        assert st["attempted"] == st_e["attempted"] and st["failed"] == st_e["failed"]
        assert st["tail_queries"] == st_e["tail_queries"]
    # other outputs: captured again, same result
    gi2, gd2 = idx.self_join(K, use_graph=1, **opts)
    gi2, gd2 = idx.self_join(K, ids=gi2, dists=gd2, use_graph=1, **opts)
    torch.cuda.synchronize()
    assert (gi2.cpu().numpy() == ref_i).all() and (gd2.cpu().numpy() == ref_d).all()
    if name == "expo3d_tail":
        assert st_e["tail_queries"] > 0 and st_e["levels"] >= 2
    idx.close()


@pytest.mark.parametrize("heavy_min", [1, 150, -1])
@pytest.mark.parametrize("name,gen,K", [
    ("expo4d", lambda: datagen.exponential(15013, 4, seed=41), 24),
    ("clus2d", lambda: datagen.clustered(20011, seed=42), 40),
    ("unif6d", lambda: datagen.uniform(4001, 6, seed=43), 5),
], ids=["expo4d", "clus2d", "unif6d"])
def test_heavy_queries(knn, oracle_mod, name, gen, K, heavy_min):
    """Queries routed to the workgroup-per-query kernel (all of them with
    heavy_min=1, the larger cells with 150, none with -1) give the oracle's
    result; with a small cell side the refinement and the failures go through
    it too."""
    D = gen()
    N = D.shape[0]
    _say(f"[heavy] {name} N={N} K={K} heavy_min={heavy_min}")
    ids, dists, st = _join(knn, D, K, heavy_min=heavy_min, w_factor=0.6, tail_pairs=-1)
    _check_rows(D, ids, dists, K, np.arange(N), oracle_mod)
    assert st["levels"] >= 2
    if heavy_min == 1:  # every searched query of every level went to the workgroup kernel
        L = st["levels"]
        assert st["heavy_queries"] == [st["attempted"][i] - st["deferred"][i] for i in range(L)]
        assert st["heavy_failed"] == [st["failed"][i] - st["deferred"][i] for i in range(L)]
    if heavy_min == -1:
        assert not any(st["heavy_queries"])


@pytest.mark.parametrize("speculate", [0, -1])
@pytest.mark.parametrize("name,gen,K,lanes", [
    ("expo4d_k24", lambda: datagen.exponential(9000, 4, seed=61), 24, 8),
    ("unif6d_k16", lambda: datagen.uniform(7000, 6, seed=62), 16, 16),
    ("expo2d_k40", lambda: datagen.exponential(8000, 2, seed=63), 40, 8),
    ("unif3d_k7", lambda: datagen.uniform(6000, 3, seed=64), 7, 4),
], ids=["expo4d_k24", "unif6d_k16", "expo2d_k40", "unif3d_k7"])
def test_speculation(knn, oracle_mod, speculate, name, gen, K, lanes):
    """Survivors kept during the count pass (collect pass skipped when they
    hold the K nearest) or always collected: the oracle's result either way,
    and with speculation on, some queries of the first level speculate."""
    D = gen()
    _say(f"[spec] {name} speculate={speculate} lanes={lanes}")
    ids, dists, st = _join(knn, D, K, speculate=speculate, lanes_per_query=lanes, tail_pairs=-1)
    _check_rows(D, ids, dists, K, np.arange(D.shape[0]), oracle_mod)
    if speculate < 0:
        assert not any(st["spec_queries"])
    else:
        assert 0 < st["spec_queries"][0] <= st["attempted"][0] - st["failed"][0]


@pytest.mark.parametrize("predict_fail", [0, -1])
@pytest.mark.parametrize("name,gen,K", [
    ("expo4d_k24", lambda: datagen.exponential(12000, 4, seed=71), 24),
    ("expo2d_k6", lambda: datagen.exponential(12000, 2, seed=72), 6),
    ("unif5d_k10", lambda: datagen.uniform(8000, 5, seed=73), 10),
], ids=["expo4d_k24", "expo2d_k6", "unif5d_k10"])
def test_predicted_failures(knn, oracle_mod, predict_fail, name, gen, K):
    """Queries whose predicted K-th distance is well beyond their covered
    radius deferred to the next level without a count pass, or all searched:
    the oracle's result either way; deferred queries count as failed."""
    D = gen()
    _say(f"[defer] {name} predict_fail={predict_fail}")
    ids, dists, st = _join(knn, D, K, predict_fail=predict_fail, w_factor=0.7, tail_pairs=-1)
    _check_rows(D, ids, dists, K, np.arange(D.shape[0]), oracle_mod)
    for L in range(st["levels"]):
        assert st["deferred"][L] <= st["failed"][L]
    if predict_fail < 0:
        assert not any(st["deferred"])
    else:
        assert st["deferred"][0] > 0


@pytest.mark.parametrize("share", [1, -1])
@pytest.mark.parametrize("name,gen,K,lanes", [
    ("unif6d_t4", lambda: datagen.uniform(6000, 6, seed=51), 12, 4),
    ("expo4d_t8", lambda: datagen.exponential(9000, 4, seed=52), 20, 8),
    ("clus2d_t2", lambda: datagen.clustered(8000, seed=53), 9, 2),
], ids=["unif6d_t4", "expo4d_t8", "clus2d_t2"])
def test_shared_lists(knn, oracle_mod, share, name, gen, K, lanes):
    """Wavefronts whose queries share a cell walking one (union) list, or each
    query its own: the oracle's result either way."""
    D = gen()
    _say(f"[share] {name} share={share} lanes={lanes}")
    ids, dists, st = _join(knn, D, K, share_lists=share, lanes_per_query=lanes)
    _check_rows(D, ids, dists, K, np.arange(D.shape[0]), oracle_mod)
