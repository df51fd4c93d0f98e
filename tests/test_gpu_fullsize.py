"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times (default options, device inputs and outputs).

Sampled rows are checked one by one against the brute-force oracle (ids
identical, distances bit-identical); every row is checked for properties that
hold at any size (ids distinct and not the point itself, distances
non-decreasing, each distance equal to the recomputed one)."""

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

pytestmark = pytest.mark.gpu

WORKLOADS = [
    ("unif2d_50k", [5]),
    ("expo2d_2m", [1, 8, 32, 64]),
    ("expo4d_2m", [1, 8, 32, 64]),
    ("unif6d_5m", [32]),
    ("clustered2d_20m", [16]),
]


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04758_amd import api
    api.load()
    return api


def _recompute_ok(Dd, ids, dists):
    """All-row properties on the GPU (torch used only to check)."""
    import torch
    N, K = ids.shape
    rows = torch.arange(N, device=ids.device, dtype=torch.int64)
    assert bool((ids.to(torch.int64) != rows[:, None]).all()), "a point is its own neighbour"
    if K > 1:
        assert bool((dists[:, 1:] >= dists[:, :-1]).all()), "distances not sorted"
        s, _ = torch.sort(ids, dim=1)
        assert bool((s[:, 1:] != s[:, :-1]).all()), "repeated neighbour"
    # distance recomputed left to right over the dimensions, one op per kernel
    step = max(1, (1 << 26) // max(1, K))
    for r0 in range(0, N, step):
        r1 = min(N, r0 + step)
        nb = ids[r0:r1].to(torch.int64)
        acc = torch.zeros((r1 - r0, K), dtype=torch.float64, device=ids.device)
        for j in range(Dd.shape[1]):
            t = Dd[nb, j] - Dd[r0:r1, j][:, None]
            acc = acc + t * t
        assert bool((torch.sqrt(acc) == dists[r0:r1]).all()), "distance differs from recomputation"


@pytest.mark.parametrize("name,Ks", WORKLOADS, ids=[w[0] for w in WORKLOADS])
def test_fullsize_sampled_parity(api, oracle_mod, name, Ks):
    import torch
    D, _, _ = datagen.config_points(name)
    N = D.shape[0]
    print(f"[fullsize] {name} N={N} K={Ks}", flush=True)
    Dd = torch.from_numpy(D).cuda()
    idx = api.build_index(Dd)
    rng = np.random.default_rng(123)
    n_rows = 64 if N > 10_000_000 else (128 if N > 1_000_000 else 256)
    rows = np.unique(np.concatenate([rng.choice(N, size=n_rows, replace=False), [0, N - 1]]))
    for K in Ks:
        ids, dists, st = idx.self_join(K, with_stats=True)
        torch.cuda.synchronize()
        print(f"  K={K} levels={st['levels']} tail={st['tail_queries']} "
              f"ms={st['ms_total']:.1f}", flush=True)
        _recompute_ok(Dd, ids, dists)
        got_i = ids[torch.from_numpy(rows).cuda()].cpu().numpy()
        got_d = dists[torch.from_numpy(rows).cuda()].cpu().numpy()
        ref_i, ref_d = oracle_mod.knn(D, K, rows=rows)
        bad = np.nonzero((got_i != ref_i).any(axis=1) | (got_d != ref_d).any(axis=1))[0]
        assert bad.size == 0, f"{bad.size} sampled rows differ, e.g. row {rows[bad[0]]}"
        del ids, dists
    idx.close()
