"""The distance similarity self-join (every pair within eps; the range-query
join of Sec. 1 / Sec. 3 that the KNN join is built from) through the C ABI,
against the oracle's eps_join (the definition, by brute force): the same set
of (query, neighbour) pairs and bit-identical distances, per-point counts
identical, batches that respect their capacity and together hold every pair
once, the host streaming path on 1-3 streams, and the edge cases (eps 0 with
duplicates, pairs exactly at eps, eps above the diameter, underflowing
squares, a capacity below one query's pairs, a consumer that stops)."""

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


def _sorted_triples(q, j, d):
    q = np.asarray(q, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    o = np.lexsort((j, q))
    return q[o], j[o], np.asarray(d)[o]


def _same_pairs(got, want):
    gq, gj, gd = _sorted_triples(*got)
    wq, wj, wd = _sorted_triples(*want)
    assert gq.size == wq.size, f"{gq.size} pairs, oracle {wq.size}"
    assert np.array_equal(gq, wq) and np.array_equal(gj, wj), "pair sets differ"
    bad = np.nonzero(gd != wd)[0]
    assert bad.size == 0, (f"{bad.size} distances differ; first ({gq[bad[0]]}, {gj[bad[0]]}): "
                           f"{gd[bad[0]]!r} vs {wd[bad[0]]!r}")


def _unif_eps(N, n, m):
    # eps holding about m points of a uniform [0,100)^n set of N points
    from math import gamma, pi
    vn = pi ** (n / 2) / gamma(n / 2 + 1)
    return 100.0 * (m / (N * vn)) ** (1.0 / n)


CASES = [
    # (name, points, eps)
    ("unif2d", lambda: datagen.uniform(6000, 2, seed=31), _unif_eps(6000, 2, 20)),
    ("expo2d", lambda: datagen.exponential(8000, 2, seed=32), 0.002),
    ("clus2d", lambda: datagen.clustered(9000, seed=33), 2.0),
    ("unif3d", lambda: datagen.uniform(6000, 3, seed=34), _unif_eps(6000, 3, 25)),
    ("expo4d", lambda: datagen.exponential(5000, 4, seed=35), 0.015),
    ("unif5d", lambda: datagen.uniform(4000, 5, seed=36), _unif_eps(4000, 5, 12)),
    ("unif6d", lambda: datagen.uniform(4000, 6, seed=37), _unif_eps(4000, 6, 10)),
    ("dyadic3d_exact", lambda: datagen.dyadic(5000, 3, seed=38, bits=3, span=8), 0.5),
    ("lattice2d_eps1", lambda: datagen.lattice(60, 2), 1.0),
    ("lattice4d_eps1", lambda: datagen.lattice(8, 4), 1.0),
    ("dups_eps0", lambda: np.concatenate([datagen.uniform(500, 3, seed=39)] * 4), 0.0),
    ("all_pairs", lambda: datagen.uniform(300, 2, seed=40), 1000.0),
    ("underflow", lambda: np.stack([np.arange(9) * 1e-170, np.zeros(9)], axis=1), 1e-200),
    ("two_points", lambda: np.array([[0.0, 0.0], [3.0, 4.0]]), 5.0),
]


@pytest.mark.parametrize("name,D,eps", CASES, ids=[c[0] for c in CASES])
def test_eps_join_every_pair(knn, oracle_mod, name, D, eps):
    import torch
    D = D()
    _say(f"[epsjoin] {name} N={D.shape[0]} n={D.shape[1]} eps={eps!r}")
    want = oracle_mod.eps_join(D, eps)
    idx = knn.build_index(torch.from_numpy(D).cuda())
    total, counts = idx.eps_join_size(eps, counts=True)
    torch.cuda.synchronize()
    assert total == want[0].size
    assert np.array_equal(counts.cpu().numpy().astype(np.int64), want[3])
    q, j, d = idx.eps_join_device(eps)
    torch.cuda.synchronize()
    _same_pairs((q.cpu().numpy(), j.cpu().numpy(), d.cpu().numpy()), want[:3])
    idx.close()


@pytest.mark.parametrize("extra", [0, 1, 997, 25000])
def test_eps_join_batches(knn, oracle_mod, extra):
    """Batches of at most cap = (the largest pair count of a query) + extra
    pairs from cursor 0 to N: whole queries each, queries contiguous, every
    pair once, and a cursor of N yields nothing."""
    import torch
    D = datagen.exponential(7000, 3, seed=41)
    eps = 0.008
    want = oracle_mod.eps_join(D, eps)
    cap = int(want[3].max()) + extra
    idx = knn.build_index(torch.from_numpy(D).cuda())
    dev = torch.device("cuda", 0)
    bq = torch.empty(cap, dtype=torch.int32, device=dev)
    bj = torch.empty(cap, dtype=torch.int32, device=dev)
    bd = torch.empty(cap, dtype=torch.float64, device=dev)
    cursor, parts, seen, nb = 0, [], set(), 0
    _say(f"[epsjoin] batches cap={cap}")
    while cursor < idx.N:
        n, nxt = idx.eps_join_batch(eps, cursor, bq, bj, bd)
        torch.cuda.synchronize()
        nb += 1
        assert nxt > cursor and n <= cap
        q = bq[:n].cpu().numpy()
        # the batch's queries: whole, contiguous, never seen before
        if n:
            starts = np.concatenate([[0], np.nonzero(np.diff(q))[0] + 1])
            qs = q[starts].tolist()
            assert len(set(qs)) == len(qs)
            assert not (set(qs) & seen)
            seen |= set(qs)
            for a, b in zip(starts, np.concatenate([starts[1:], [n]])):
                assert b - a == want[3][q[a]]
        parts.append((q, bj[:n].cpu().numpy(), bd[:n].cpu().numpy()))
        cursor = nxt
    assert cursor == idx.N
    assert nb >= -(-want[0].size // cap)
    got = tuple(np.concatenate([p[i] for p in parts]) for i in range(3))
    _same_pairs(got, want[:3])
    assert idx.eps_join_batch(eps, idx.N, bq, bj, bd) == (0, idx.N)
    idx.close()


def test_eps_join_capacity_below_one_query(knn, oracle_mod):
    """A capacity below the pairs of the query at the cursor is an error that
    names the count; the cursor does not move, and a larger capacity goes on."""
    import torch
    D = datagen.uniform(3000, 2, seed=47)
    eps = _unif_eps(3000, 2, 15)
    want = oracle_mod.eps_join(D, eps)
    idx = knn.build_index(torch.from_numpy(D).cuda())
    dev = torch.device("cuda", 0)
    cap = int(want[3].max()) - 1
    bq = torch.empty(cap + 1, dtype=torch.int32, device=dev)
    bj = torch.empty(cap + 1, dtype=torch.int32, device=dev)
    bd = torch.empty(cap + 1, dtype=torch.float64, device=dev)
    cursor, failed = 0, False
    while cursor < idx.N:
        try:
            n, cursor = idx.eps_join_batch(eps, cursor, bq[:cap], bj[:cap], bd[:cap])
        except knn._lib.KnnError as e:
            assert e.code == knn._lib.KNN_EINVAL and f"the {cap + 1} pairs" in str(e)
            failed = True
            n, nxt = idx.eps_join_batch(eps, cursor, bq, bj, bd)
            assert nxt > cursor
            cursor = nxt
    assert failed
    idx.close()


def test_eps_join_estimate(knn):
    """The sampled size estimate: exact at stride 1, within 10 % on a
    uniform set at strides 4 and 16, and a valid count for a stride above N."""
    import torch
    D = datagen.uniform(40000, 2, seed=42)
    eps = _unif_eps(40000, 2, 30)
    idx = knn.build_index(torch.from_numpy(D).cuda())
    exact = idx.eps_join_size(eps)
    _say(f"[epsjoin] estimate exact={exact}")
    for s in (4, 16):
        est = idx.eps_join_size(eps, sample_stride=s)
        assert abs(est - exact) <= 0.1 * exact, (s, est, exact)
    assert idx.eps_join_size(eps, sample_stride=10 ** 9) >= 0
    # batches after an estimate still use exact counts
    q, j, d = idx.eps_join_device(eps, capacity=500000)
    assert q.numel() == exact
    idx.close()


@pytest.mark.parametrize("streams,batch", [(1, 5000), (2, 777), (3, 20000), (0, 0)])
def test_eps_join_host_streaming(knn, oracle_mod, streams, batch):
    """knn_eps_join: batches copied to pinned host buffers while the next ones
    run on `streams` streams, handed over in order; together every pair."""
    import torch
    D = datagen.clustered(12000, seed=43)
    eps = 2.0
    want = oracle_mod.eps_join(D, eps)
    if batch:
        batch = max(batch, int(want[3].max()))  # every query fits a batch
    idx = knn.build_index(torch.from_numpy(D).cuda())
    _say(f"[epsjoin] host streams={streams} batch={batch}")
    q, j, d, st = idx.eps_join(eps, batch_pairs=batch, n_streams=streams)
    assert st["n_pairs"] == want[0].size
    if batch:
        assert st["n_batches"] >= -(-want[0].size // batch)
    _same_pairs((q, j, d), want[:3])
    # batches arrive in cursor order: the same sequence as the device batches
    dq, dj, dd = idx.eps_join_device(eps, capacity=batch or want[0].size)
    assert np.array_equal(q, dq.cpu().numpy()) and np.array_equal(j, dj.cpu().numpy())
    idx.close()


def test_eps_join_consumer_stops(knn):
    import torch
    D = datagen.uniform(5000, 2, seed=44)
    idx = knn.build_index(torch.from_numpy(D).cuda())
    calls = []

    def stop_second(q, j, d):
        calls.append(q.size)
        return len(calls) == 2

    with pytest.raises(knn._lib.KnnError) as ei:
        idx.eps_join(2.0, consume=stop_second, batch_pairs=2000, n_streams=3)
    assert ei.value.code == knn._lib.KNN_ECANCELED
    assert len(calls) == 2
    # the index is usable afterwards
    assert idx.eps_join_size(2.0) > 0
    idx.eps_join_release()
    idx.close()


def test_eps_join_invalid(knn):
    import torch
    idx = knn.build_index(torch.from_numpy(datagen.uniform(100, 2, seed=45)).cuda())
    for eps in (-1.0, float("nan"), float("inf")):
        with pytest.raises(knn._lib.KnnError) as ei:
            idx.eps_join_size(eps)
        assert ei.value.code == knn._lib.KNN_EINVAL
    with pytest.raises(knn._lib.KnnError):
        idx.eps_join_size(1.0, sample_stride=0)
    dev = torch.device("cuda", 0)
    b = torch.empty(4, dtype=torch.int32, device=dev)
    bd = torch.empty(4, dtype=torch.float64, device=dev)
    with pytest.raises(knn._lib.KnnError):
        idx.eps_join_batch(1.0, idx.N + 1, b, b.clone(), bd)
    idx.close()


def test_eps_join_then_knn(knn, oracle_mod):
    """The eps join's state and a KNN join on the same index do not disturb
    each other, and eps_join's counts at eps_min(K) relate to the KNN rows:
    a point with at least K pairs within eps has its K-th distance <= eps."""
    import torch
    D = datagen.exponential(6000, 2, seed=46)
    idx = knn.build_index(torch.from_numpy(D).cuda())
    K = 8
    eps = idx.eps_min(K)
    total, counts = idx.eps_join_size(eps, counts=True)
    ids, dists = idx.self_join(K)
    q, j, d = idx.eps_join_device(eps)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    kth = dists.cpu().numpy()[:, K - 1]
    assert np.all(kth[c >= K] <= eps)
    assert np.all(kth[c < K] > eps)
    want = oracle_mod.eps_join(D, eps)
    _same_pairs((q.cpu().numpy(), j.cpu().numpy(), d.cpu().numpy()), want[:3])
    ref_i, ref_d = oracle_mod.knn(D, K)
    assert np.array_equal(ids.cpu().numpy(), ref_i)
    idx.close()
