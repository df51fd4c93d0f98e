"""GPU tests of the serving loop (knn_server_*): continuous batching over
resident indexes, memory admission, and bit-identical results alone and in
the mix."""

import sys

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04758_amd import api
    api.load()
    return api


def _datasets():
    return [
        datagen.uniform(12000, 2, seed=70),
        datagen.exponential(9000, 3, seed=71),
        datagen.uniform(7000, 4, seed=72),
        datagen.exponential(5000, 6, seed=73),
        datagen.clustered(15000, seed=74),
    ]


def test_mix_equals_solo_and_oracle(api, oracle_mod):
    print("[serving] mix vs solo", flush=True)
    Ds = _datasets()
    idxs = [api.build_index(D) for D in Ds]
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(len(Ds))), int(rng.choice([1, 4, 16, 64]))) for _ in range(24)]
    # solo results (one join at a time on the index's own context)
    solo = {}
    for ds, K in set(reqs):
        solo[(ds, K)] = idxs[ds].self_join_host(K)
    srv = api.Server(mem_budget_bytes=1 << 30, max_inflight=4)
    ids_ = [srv.add_dataset(ix) for ix in idxs]
    assert ids_ == list(range(len(Ds)))
    tickets = [(srv.submit(ds, K, Ds[ds].shape[0]), ds, K) for ds, K in reqs]
    for t, ds, K in tickets:
        got_ids, got_d = srv.wait(t)
        ref_ids, ref_d = solo[(ds, K)]
        assert (got_ids == ref_ids).all() and (got_d == ref_d).all()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"] + 1e-9
    assert st["peak_inflight"] >= 2  # requests overlapped on the device
    assert st["peak_bytes"] <= 1 << 30
    srv.close()
    # the solo results themselves match the oracle on sampled rows
    for (ds, K), (ids, d) in solo.items():
        rows = np.arange(0, Ds[ds].shape[0], 97)
        r_ids, r_d = oracle_mod.knn(Ds[ds], K, rows=rows)
        assert (ids[rows] == r_ids).all() and (d[rows] == r_d).all()
    for ix in idxs:
        ix.close()


def test_admission_budget(api):
    print("[serving] admission", flush=True)
    from paper_1810_04758_amd._lib import KnnError, KNN_EINVAL
    D = datagen.uniform(20000, 2, seed=75)
    ix = api.build_index(D)
    # a budget that fits one request at a time: requests queue, never fail
    fp = ix.join_footprint(8)
    budget = int(fp * 1.5)
    srv = api.Server(mem_budget_bytes=budget, max_inflight=4)
    ds = srv.add_dataset(ix)
    ts = [srv.submit(ds, 8, D.shape[0]) for _ in range(6)]
    outs = [srv.wait(t) for t in ts]
    for ids, d in outs[1:]:
        assert (ids == outs[0][0]).all() and (d == outs[0][1]).all()
    st = srv.stats()
    assert st["completed"] == 6
    assert st["peak_bytes"] <= budget
    assert st["peak_inflight"] == 1
    # a request larger than the whole budget is rejected
    with pytest.raises(KnnError) as e:
        srv.submit(ds, 1024, D.shape[0])
    assert e.value.code == KNN_EINVAL
    srv.close()
    ix.close()


def test_wait_timeout_and_unknown_ticket(api):
    from paper_1810_04758_amd._lib import KnnError
    D = datagen.uniform(3000, 2, seed=76)
    ix = api.build_index(D)
    srv = api.Server(max_inflight=2)
    ds = srv.add_dataset(ix)
    t = srv.submit(ds, 4, D.shape[0])
    srv.wait(t)
    with pytest.raises(KnnError):
        srv.wait(t)  # already collected
    srv.close()
    ix.close()


@pytest.mark.parametrize("name,gen,K,opts", [
    # small cells at level 0 (row table), larger ones later (dense key table):
    # a context once held both
    ("expo3d_levels", lambda: datagen.exponential(200_000, 3, seed=77), 8, {"w_factor": 0.25}),
    ("unif2d", lambda: datagen.uniform(100_000, 2, seed=78), 16, {}),
    ("unif6d", lambda: datagen.uniform(30_000, 6, seed=79), 8, {"w_factor": 0.5}),
])
def test_footprint_bounds_what_a_join_holds(api, name, gen, K, opts):
    """knn_join_footprint (the admission size) is an upper bound of the device
    memory a join with host outputs actually holds, device cache slack
    included, also for a join that runs many levels."""
    print(f"[serving] footprint {name}", flush=True)
    D = gen()
    ix = api.build_index(D)
    before = ix.info()["device_bytes"]  # the index alone (no join scratch yet)
    fp = ix.join_footprint(K)
    _, _, st = ix.self_join_host(K, with_stats=True, **opts)
    held = ix.info()["device_bytes"] - before
    assert st["levels"] >= 2 or name == "unif2d"
    assert 0 < held <= fp, (held, fp)
    ix.close()
