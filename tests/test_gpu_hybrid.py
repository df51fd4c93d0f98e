"""The hybrid CPU/GPU KNN self-join (Sec. 4.1-4.5) through the C ABI against
the oracle's brute-force definition: every row identical (ids, and
distances bit for bit) whichever side solved it, with the GPU taking
monolithic and small batches from the dense end of the work queue, its
failures going back to the queue, and host threads taking the sparse end
with their kd-tree; plus the bookkeeping (every query solved once, the
load-imbalance metric in [0, 1], the kd-tree kept between calls) and the
argument errors."""

import sys

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

pytestmark = pytest.mark.gpu


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


def _check_rows(D, K, ids, dists, oracle_mod):
    ref_i, ref_d = oracle_mod.knn(D, K)
    bad = np.nonzero((ids != ref_i).any(axis=1) | (dists != ref_d).any(axis=1))[0]
    assert bad.size == 0, (f"{bad.size} rows differ; first {bad[0]}: got {ids[bad[0]].tolist()} "
                           f"{dists[bad[0]].tolist()} want {ref_i[bad[0]].tolist()} "
                           f"{ref_d[bad[0]].tolist()}")


def _check_stats(st, N, eps_factor=1.0):
    assert st["gpu_queries"] + st["cpu_queries"] == N
    assert st["gpu_attempts"] >= st["gpu_queries"]
    assert 0.0 <= st["load_imbalance"] <= 1.0
    # eps starts at eps_factor * eps_min and grows by eps_min / 2 per re-index
    e0 = eps_factor * st["eps_min"]
    assert st["ms_total"] > 0
    assert abs(st["eps_final"] - (e0 + 0.5 * st["eps_min"] * st["reindexes"])) <= 1e-9 * st["eps_final"]


CASES = [
    # (name, points, K)
    ("unif2d", lambda: datagen.uniform(20000, 2, seed=51), 8),
    ("expo2d", lambda: datagen.exponential(30000, 2, seed=52), 16),
    ("clus2d", lambda: datagen.clustered(30000, seed=53), 12),
    ("expo3d", lambda: datagen.exponential(12000, 3, seed=54), 9),
    ("expo4d", lambda: datagen.exponential(8000, 4, seed=55), 5),
    ("unif6d", lambda: datagen.uniform(5000, 6, seed=56), 10),
    ("dups2d", lambda: np.concatenate([datagen.uniform(800, 2, seed=57)] * 6), 9),
    ("kN", lambda: datagen.uniform(200, 3, seed=58), 199),
]

MODES = [
    # (name, options)
    ("default", dict(cpu_threads=4)),
    # tiny GPU batches and a small first eps: the host threads get much of
    # the queue, and the GPU hands many failures back
    ("cpu_heavy", dict(cpu_threads=6, n_large=-1.0, n_small=0.002, n_cpu=0.002,
                       eps_factor=0.3)),
    ("gpu_only", dict(cpu_threads=-1)),
]


@pytest.mark.parametrize("mode,opts", MODES, ids=[m[0] for m in MODES])
@pytest.mark.parametrize("name,D,K", CASES, ids=[c[0] for c in CASES])
def test_hybrid_every_row(knn, oracle_mod, name, D, K, mode, opts):
    import torch
    D = D()
    N = D.shape[0]
    idx = knn.build_index(torch.from_numpy(D).cuda())
    _say(f"[hybrid] {name} N={N} n={D.shape[1]} K={K} mode={mode}")
    ids, dists, st = idx.self_join_hybrid(K, **opts)
    _say(f"  gpu {st['gpu_queries']} cpu {st['cpu_queries']} batches {st['gpu_batches']} "
         f"(monolithic {st['monolithic_batches']}) reindexes {st['reindexes']} "
         f"imbalance {st['load_imbalance']:.3f}")
    _check_stats(st, N, opts.get("eps_factor", 1.0))
    if mode == "gpu_only":
        assert st["cpu_queries"] == 0 and st["load_imbalance"] == 0.0
    if mode == "cpu_heavy" and N >= 5000:
        assert st["cpu_queries"] > 0
    _check_rows(D, K, ids, dists, oracle_mod)
    idx.close()


def test_hybrid_schedule_and_reuse(knn, oracle_mod):
    """Monolithic rounds happen when n_large > 0 and none when it is off; a
    second call reuses the kd-tree (no build time) and gives the same rows."""
    import torch
    D = datagen.exponential(40000, 2, seed=59)
    K = 8
    idx = knn.build_index(torch.from_numpy(D).cuda())
    ids1, d1, st1 = idx.self_join_hybrid(K, cpu_threads=4)
    assert st1["monolithic_batches"] >= 1 and st1["ms_cpu_index"] > 0
    ids2, d2, st2 = idx.self_join_hybrid(K, cpu_threads=4)
    assert st2["ms_cpu_index"] == 0
    assert np.array_equal(ids1, ids2) and np.array_equal(d1, d2)
    _, _, st3 = idx.self_join_hybrid(K, cpu_threads=-1, n_large=-1.0, n_small=0.05)
    assert st3["monolithic_batches"] == 0 and st3["gpu_batches"] >= 20
    # a GPU-only run whose first eps is tiny: many failures, eps grows
    ids4, d4, st4 = idx.self_join_hybrid(K, cpu_threads=-1, eps_factor=0.05)
    assert st4["reindexes"] >= 1 and st4["gpu_attempts"] > D.shape[0]
    _check_rows(D, K, ids4, d4, oracle_mod)
    # the hybrid leaves the index's other joins intact
    gi, gd = idx.self_join(K)
    assert np.array_equal(gi.cpu().numpy(), ids1)
    idx.close()


def test_hybrid_invalid(knn):
    import torch
    idx = knn.build_index(torch.from_numpy(datagen.uniform(300, 2, seed=60)).cuda())
    for K in (0, 300, 1024):
        with pytest.raises(knn._lib.KnnError) as ei:
            idx.self_join_hybrid(K)
        assert ei.value.code == knn._lib.KNN_EINVAL
    idx.close()
