"""The KNN join of a query set with the indexed set (R join_KNN S, Sec. 2.1;
the query set of the GPU kernel, Sec. 4.3) through the C ABI, against the
oracle's knn_rs (brute force by the definition): ids identical and distances
bit-identical on every row.  Queries drawn from the indexed set's
distribution, copies of indexed points (distance-0 neighbours, nothing
excluded), queries far outside the indexed set's box, duplicates, K = N;
both level structures, many levels, the tail and the heavy-query kernel."""

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


def _rows_equal(S, Q, ids, dists, K, oracle_mod, rows=None):
    ref_i, ref_d = oracle_mod.knn_rs(S, Q, K, rows=rows)
    if rows is not None:
        ids, dists = ids[rows], dists[rows]
    bad = np.nonzero((ids != ref_i).any(axis=1) | (dists != ref_d).any(axis=1))[0]
    assert bad.size == 0, (f"{bad.size} rows differ; first {bad[0]}: got {ids[bad[0]].tolist()} "
                           f"{dists[bad[0]].tolist()} want {ref_i[bad[0]].tolist()} "
                           f"{ref_d[bad[0]].tolist()}")


def _far(n, seed):
    return datagen.uniform(40, n, seed=seed) * 30 + 500.0


CASES = [
    # (name, S, Q, K)
    ("unif2d", lambda: datagen.uniform(4000, 2, seed=1), lambda: datagen.uniform(3001, 2, seed=2), 7),
    ("expo2d_copies", lambda: datagen.exponential(5000, 2, seed=3),
     lambda: np.concatenate([datagen.exponential(2000, 2, seed=4),
                             datagen.exponential(5000, 2, seed=3)[::7]]), 16),
    ("clus2d_far", lambda: datagen.clustered(6000, seed=5),
     lambda: np.concatenate([datagen.clustered(2500, seed=6), _far(2, 7)]), 12),
    ("expo3d", lambda: datagen.exponential(4000, 3, seed=8), lambda: datagen.exponential(2500, 3, seed=9), 9),
    ("unif4d_far", lambda: datagen.uniform(3000, 4, seed=10),
     lambda: np.concatenate([datagen.uniform(1500, 4, seed=11), _far(4, 12)]), 5),
    ("unif5d", lambda: datagen.uniform(2500, 5, seed=13), lambda: datagen.uniform(1200, 5, seed=14), 6),
    ("unif6d", lambda: datagen.uniform(3000, 6, seed=15), lambda: datagen.uniform(900, 6, seed=16), 10),
    ("dups2d", lambda: np.concatenate([datagen.uniform(300, 2, seed=17)] * 5),
     lambda: datagen.uniform(400, 2, seed=18), 12),
    ("kN", lambda: datagen.uniform(150, 3, seed=19), lambda: datagen.uniform(60, 3, seed=20), 150),
    ("tiny", lambda: np.array([[0.0, 0.0], [1.0, 2.0]]), lambda: np.array([[0.4, 0.9]]), 2),
]


@pytest.mark.parametrize("name,S,Q,K", CASES, ids=[c[0] for c in CASES])
def test_join_every_row(knn, oracle_mod, name, S, Q, K):
    import torch
    S, Q = S(), Q()
    idx = knn.build_index(torch.from_numpy(S).cuda())
    Qd = torch.from_numpy(Q).cuda()
    structures = [-1, 1] if S.shape[1] <= 4 else [0]
    for z in structures:
        for wf in (0.25, 1.0):
            _say(f"[rjoin] {name} N={S.shape[0]} NQ={Q.shape[0]} n={S.shape[1]} K={K} "
                 f"zorder={z} w_factor={wf}")
            ids, dists, st = idx.join(Qd, K, with_stats=True, zorder=z, w_factor=wf)
            torch.cuda.synchronize()
            _rows_equal(S, Q, ids.cpu().numpy(), dists.cpu().numpy(), K, oracle_mod)
    idx.close()


@pytest.mark.parametrize("opts", [
    dict(tail_pairs=1e15),                 # every failure of level 0 to the tail
    dict(tail_pairs=-1.0, w_factor=0.05),  # many levels, no tail
    dict(heavy_min=8, tail_pairs=-1.0),    # the heavy-query kernel
    dict(schedule=1, batch_queries=700),
    dict(predict_fail=-1, speculate=-1),
    dict(lanes_per_query=64),
], ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()))
@pytest.mark.parametrize("z", [-1, 1])
def test_join_options(knn, oracle_mod, opts, z):
    import torch
    S = datagen.exponential(6000, 2, seed=21)
    Q = np.concatenate([datagen.exponential(3000, 2, seed=22), S[:100], _far(2, 23)])
    K = 20
    _say(f"[rjoin options] zorder={z} {opts}")
    idx = knn.build_index(torch.from_numpy(S).cuda())
    ids, dists, st = idx.join(torch.from_numpy(Q).cuda(), K, with_stats=True, zorder=z, **opts)
    torch.cuda.synchronize()
    idx.close()
    _rows_equal(S, Q, ids.cpu().numpy(), dists.cpu().numpy(), K, oracle_mod)
    if opts.get("tail_pairs") == 1e15:
        assert st["tail_queries"] > 0
    if "heavy_min" in opts:
        assert sum(st["heavy_queries"][:st["levels"]]) > 0


def test_join_host_entry_and_self_relation(knn, oracle_mod):
    """knn_join with host arrays; and Q = D: each row holds the point itself
    at distance 0 (behind lower-id duplicates), the rest is the self-join's."""
    D = np.concatenate([datagen.uniform(2000, 3, seed=24), datagen.uniform(2000, 3, seed=24)[:50]])
    K = 9
    idx = knn.build_index(D)
    ids, dists = idx.join(D, K + 1)
    si, sd = idx.self_join_host(K)
    idx.close()
    _rows_equal(D, D, ids, dists, K + 1, oracle_mod)
    for i in range(0, D.shape[0], 13):
        row = ids[i].tolist()
        assert i in row and dists[i, row.index(i)] == 0.0
        assert [j for j in row if j != i][:K] == si[i].tolist()


def test_join_larger_sampled(knn, oracle_mod):
    """2e5 clustered indexed points, 1e5 queries of another draw (and a few
    far ones): random rows and the sparsest queries (largest K-th distance)
    against the oracle."""
    import torch
    S = datagen.clustered(200_000, seed=25)
    Q = np.concatenate([datagen.clustered(100_000, seed=26), _far(2, 27)])
    K = 16
    _say(f"[rjoin sized] N={S.shape[0]} NQ={Q.shape[0]}")
    idx = knn.build_index(torch.from_numpy(S).cuda())
    for z in (-1, 1):
        ids, dists, st = idx.join(torch.from_numpy(Q).cuda(), K, with_stats=True, zorder=z)
        torch.cuda.synchronize()
        ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
        rng = np.random.default_rng(1)
        rows = np.unique(np.concatenate([rng.choice(Q.shape[0], 1500, replace=False),
                                         np.argsort(dists[:, -1])[-300:],
                                         np.arange(Q.shape[0] - 40, Q.shape[0])]))
        _rows_equal(S, Q, ids, dists, K, oracle_mod, rows=rows)
        _say(f"  zorder={z} levels={st['levels']} tail={st['tail_queries']} ms={st['ms_total']:.1f}")
    idx.close()


def test_join_invalid(knn):
    import torch
    from paper_1810_04758_amd._lib import KNN_EINVAL, KnnError
    S = datagen.uniform(100, 2, seed=28)
    idx = knn.build_index(S)
    Q = datagen.uniform(10, 2, seed=29)
    for bad in (dict(K=101), dict(K=0), dict(K=3, use_graph=1)):
        K = bad.pop("K")
        with pytest.raises(KnnError) as e:
            idx.join(torch.from_numpy(Q).cuda(), K, **bad)
        assert e.value.code == KNN_EINVAL
    Qn = Q.copy()
    Qn[3, 1] = np.inf
    with pytest.raises(KnnError) as e:
        idx.join(torch.from_numpy(Qn).cuda(), 3)
    assert e.value.code == KNN_EINVAL
    with pytest.raises(ValueError):
        idx.join(datagen.uniform(5, 3, seed=1), 3)
    ids, _ = idx.join(Q, 100)  # K = N: every point, ordered
    assert all(sorted(r) == list(range(100)) for r in ids.tolist())
    idx.close()


def test_host_outputs_staged_copy(knn):
    """Results above the staged-copy threshold (several 64 MiB chunks through
    the pinned double buffer) arrive in host memory identical to the device
    outputs, for the self-join and the query-set join."""
    import torch
    D = datagen.uniform(1_000_000, 2, seed=61)
    Q = datagen.uniform(700_000, 2, seed=62)
    K = 12
    idx = knn.build_index(torch.from_numpy(D).cuda())
    _say(f"[rjoin] staged host copy N={D.shape[0]} NQ={Q.shape[0]} K={K}")
    hi, hd = idx.self_join_host(K)
    di, dd = idx.self_join(K)
    torch.cuda.synchronize()
    assert np.array_equal(hi, di.cpu().numpy()) and np.array_equal(hd, dd.cpu().numpy())
    qi, qd = idx.join(Q, K)
    gi, gd = idx.join(torch.from_numpy(Q).cuda(), K)
    torch.cuda.synchronize()
    assert np.array_equal(qi, gi.cpu().numpy()) and np.array_equal(qd, gd.cpu().numpy())
    idx.close()
