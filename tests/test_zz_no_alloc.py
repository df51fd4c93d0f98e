"""The no-allocation join (knn_self_join_device_noalloc) against the ordinary
device join (knn_self_join_device) on the same index and K: neighbour ids
identical and distances bit-identical, on two calls in a row, the second with
a smaller input (the fixed scratch area keeps the first call's contents).
Also its argument checks: a join too large for the area, statistics and
graph requests are refused with KNN_EINVAL before any work."""

import sys

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04758_amd import api
    api.load()
    return api


def _both(api, D, K, **opts):
    import torch
    idx = api.build_index(torch.from_numpy(D).cuda())
    ref_i, ref_d = idx.self_join(K, **opts)
    ids = torch.full((idx.N, K), -7, dtype=torch.int32, device="cuda")
    dists = torch.full((idx.N, K), -7.0, dtype=torch.float64, device="cuda")
    idx.self_join_noalloc(K, ids, dists, **opts)
    torch.cuda.synchronize()
    out = (ref_i.cpu().numpy(), ref_d.cpu().numpy(), ids.cpu().numpy(), dists.cpu().numpy())
    idx.close()
    return out


# (name, points, K, options): each pair is run larger first, then smaller
SEQUENCES = [
    ("expo2d", lambda: datagen.exponential(60_000, 2, seed=41),
     lambda: datagen.exponential(5_003, 2, seed=42), 8, {}),
    ("unif3d_levels", lambda: datagen.uniform(40_000, 3, seed=43),
     lambda: datagen.uniform(2_999, 3, seed=44), 16, dict(w_factor=0.3)),
    ("expo4d_tail", lambda: datagen.exponential(20_000, 4, seed=45),
     lambda: datagen.exponential(1_500, 4, seed=46), 5, dict(w_factor=0.25, tail_pairs=1e9)),
    ("unif6d", lambda: datagen.uniform(6_000, 6, seed=47),
     lambda: datagen.uniform(777, 6, seed=48), 10, {}),
]


@pytest.mark.parametrize("name,big,small,K,opts", SEQUENCES, ids=[s[0] for s in SEQUENCES])
def test_noalloc_equals_device_join(api, oracle_mod, name, big, small, K, opts):
    for which, make in (("first (larger)", big), ("second (smaller)", small)):
        D = make()
        _say(f"[noalloc] {name} {which} N={D.shape[0]} n={D.shape[1]} K={K} opts={opts}")
        ri, rd, gi, gd = _both(api, D, K, **opts)
        bad = np.nonzero((gi != ri).any(axis=1) | (gd != rd).any(axis=1))[0]
        assert bad.size == 0, f"{bad.size} rows differ from the device join, e.g. row {bad[0]}"
    # the smaller input once more against the oracle itself
    oi, od = oracle_mod.knn(D, K)
    assert (gi == oi).all() and (gd == od).all()


def test_noalloc_refuses_what_it_cannot_do(api):
    import torch
    from paper_1810_04758_amd._lib import KNN_EINVAL, JoinStats, KnnError
    _say("[noalloc] argument checks")
    # a join whose buffers exceed the fixed area
    D = datagen.uniform(400_000, 2, seed=49)
    idx = api.build_index(torch.from_numpy(D).cuda())
    ids = torch.empty((idx.N, 4), dtype=torch.int32, device="cuda")
    dists = torch.empty((idx.N, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(KnnError) as e:
        idx.self_join_noalloc(4, ids, dists)
    assert e.value.code == KNN_EINVAL and "scratch" in str(e.value)
    idx.close()
    D = datagen.uniform(3_000, 2, seed=50)
    idx = api.build_index(torch.from_numpy(D).cuda())
    ids = torch.empty((idx.N, 4), dtype=torch.int32, device="cuda")
    dists = torch.empty((idx.N, 4), dtype=torch.float64, device="cuda")
    for bad in (dict(use_graph=1), dict(stats=JoinStats())):
        with pytest.raises(KnnError) as e:
            idx.self_join_noalloc(4, ids, dists, **bad)
        assert e.value.code == KNN_EINVAL
    # still usable afterwards
    idx.self_join_noalloc(4, ids, dists)
    ri, rd = idx.self_join(4)
    torch.cuda.synchronize()
    assert torch.equal(ri, ids) and torch.equal(rd, dists)
    idx.close()
