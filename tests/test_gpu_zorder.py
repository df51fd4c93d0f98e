"""Z-order levels (zorder option, 2-4 dimensions): the points are sorted once
by their bit-interleaved level-0 cell key, and each re-index doubles the cell
side by shifting that key, so every coarser cell is a run of the one sorted
order.  The grid and the level schedule change; the result may not: every row
is compared with the oracle (ids identical, distances bit-identical), and with
the row-major levels' result.  Small level-0 sides force long ladders (many
levels, the top one a single cell); the data cover clusters, duplicates, an
all-identical set, far outliers (sparse grids whose neighbour cells lie far
apart in the sorted cell table), lattices with points on cell faces, and a
zero-extent dimension."""

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


def _rows_equal_oracle(D, ids, dists, K, oracle_mod):
    ref_ids, ref_d = oracle_mod.knn(D, K)
    bad = np.nonzero((ids != ref_ids).any(axis=1) | (dists != ref_d).any(axis=1))[0]
    assert bad.size == 0, (f"{bad.size} rows differ; first row {bad[0]}: got "
                           f"{ids[bad[0]].tolist()} {dists[bad[0]].tolist()} want "
                           f"{ref_ids[bad[0]].tolist()} {ref_d[bad[0]].tolist()}")


def _join(idx, K, **opts):
    import torch
    ids, dists, st = idx.self_join(K, with_stats=True, **opts)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dists.cpu().numpy(), st


def _outliers(n):
    D = datagen.uniform(3000, n, seed=70 + n) / 100.0
    return np.concatenate([D, np.full((3, n), 1e4) + np.arange(3)[:, None]])


DATA = [
    ("unif2d", lambda: datagen.uniform(4001, 2, seed=71), 6),
    ("expo2d", lambda: datagen.exponential(5003, 2, seed=72), 16),
    ("clus2d", lambda: datagen.clustered(6007, seed=73), 16),
    ("expo3d", lambda: datagen.exponential(4003, 3, seed=74), 9),
    ("unif3d", lambda: datagen.uniform(3001, 3, seed=75), 32),
    ("expo4d", lambda: datagen.exponential(4099, 4, seed=76), 12),
    ("unif4d", lambda: datagen.uniform(2999, 4, seed=77), 5),
    ("dups2d", lambda: np.concatenate([datagen.uniform(400, 2, seed=78)] * 6), 10),
    ("same3d", lambda: np.full((600, 3), 2.5), 20),
    ("outliers2d", lambda: _outliers(2), 5),
    ("outliers3d", lambda: _outliers(3), 5),
    ("outliers4d", lambda: _outliers(4), 5),
    ("lattice2d", lambda: datagen.lattice(20, 2), 12),
    ("lattice3d", lambda: datagen.lattice(8, 3), 7),
    ("line2d", lambda: np.stack([np.linspace(0, 1, 1500) ** 2, np.zeros(1500)], 1), 6),
    ("n2", lambda: np.array([[0.0, 0.0], [1.0, 2.0]]), 1),
    ("kmax", lambda: datagen.uniform(260, 3, seed=79), 259),
]


@pytest.mark.parametrize("name,gen,K", DATA, ids=[d[0] for d in DATA])
def test_zorder_every_row(knn, oracle_mod, name, gen, K):
    import torch
    D = gen()
    idx = knn.build_index(torch.from_numpy(D).cuda())
    ref = None
    for wf in (0.03125, 0.25, 1.0, 3.0):
        _say(f"[zorder] {name} N={D.shape[0]} n={D.shape[1]} K={K} w_factor={wf}")
        ids, dists, st = _join(idx, K, zorder=1, w_factor=wf)
        if ref is None:
            _rows_equal_oracle(D, ids, dists, K, oracle_mod)
            ref = (ids, dists)
        else:
            assert (ids == ref[0]).all() and (dists == ref[1]).all()
        # cell sides double exactly from level to level
        w = np.array(st["cell_width"][:st["levels"]])
        assert (w[1:] == 2 * w[:-1]).all()
    ids, dists, _ = _join(idx, K, zorder=-1)
    assert (ids == ref[0]).all() and (dists == ref[1]).all()
    idx.close()


@pytest.mark.parametrize("opts", [
    dict(schedule=1, batch_queries=512),
    dict(lanes_per_query=2),
    dict(lanes_per_query=64),
    dict(heavy_min=16),          # most queries on the heavy kernel
    dict(tail_pairs=0.0),        # the default tail budget
    dict(tail_pairs=1e15),       # every failure of level 0 to the tail
    dict(predict_fail=-1, speculate=-1),
    dict(share_lists=1),
], ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()))
def test_zorder_options(knn, oracle_mod, opts):
    import torch
    D = datagen.exponential(5001, 2, seed=80)
    D = np.concatenate([D, D[:200]])  # duplicates
    K = 24
    _say(f"[zorder options] {opts}")
    idx = knn.build_index(torch.from_numpy(D).cuda())
    # no brute-force tail unless asked for: the ladder climbs level by level
    opts = dict(dict(tail_pairs=-1.0), **opts)
    ids, dists, st = _join(idx, K, zorder=1, w_factor=0.125, **opts)
    idx.close()
    _rows_equal_oracle(D, ids, dists, K, oracle_mod)
    if opts["tail_pairs"] == -1.0:
        assert st["tail_queries"] == 0 and st["levels"] > 2
    if "heavy_min" in opts:
        assert sum(st["heavy_queries"][:st["levels"]]) > 0


def test_zorder_graph_replay(knn, oracle_mod):
    import torch
    D = datagen.exponential(4500, 3, seed=81)
    K = 10
    _say("[zorder graph]")
    idx = knn.build_index(torch.from_numpy(D).cuda())
    ids = torch.empty((idx.N, K), dtype=torch.int32, device="cuda")
    dists = torch.empty((idx.N, K), dtype=torch.float64, device="cuda")
    eager_i, eager_d, _ = _join(idx, K, zorder=1, w_factor=0.1)
    for rep in range(4):  # capture, then replays with eager work in between
        ids.fill_(-1)
        idx.self_join(K, ids=ids, dists=dists, zorder=1, w_factor=0.1, use_graph=1)
        torch.cuda.synchronize()
        assert (ids.cpu().numpy() == eager_i).all() and (dists.cpu().numpy() == eager_d).all()
        _join(idx, K, zorder=-1)
    idx.close()
    _rows_equal_oracle(D, eager_i, eager_d, K, oracle_mod)


def test_zorder_larger_sizes_sampled(knn, oracle_mod):
    """Several tiles of every kernel and the default level-0 side: 2e5 points
    of clustered 2-D data and 1e5 of exponential 4-D data; rows checked: a
    random sample plus the sparsest and densest (by the oracle's K-th
    distance over the whole set, from its kd-tree search)."""
    import torch
    for name, D, K in (("clustered2d", datagen.clustered(200_000, seed=82), 16),
                       ("expo4d", datagen.exponential(100_000, 4, seed=83), 8)):
        _say(f"[zorder sized] {name} N={D.shape[0]} K={K}")
        idx = knn.build_index(torch.from_numpy(D).cuda())
        ids, dists, st = _join(idx, K, zorder=1)
        idx.close()
        ref_i, ref_d = oracle_mod.knn_kdtree(D, K)
        bad = np.nonzero((ids != ref_i).any(axis=1) | (dists != ref_d).any(axis=1))[0]
        assert bad.size == 0, f"{bad.size} rows differ, e.g. {bad[0]}"
        L = st["levels"]
        att, cells = st["attempted"][:L], st["cells"][:L]
        _say(f"  levels={L} tail={st['tail_queries']} attempted={att} cells={cells}")
        if name == "clustered2d":
            # a later level with few queries ran without a cell table (one
            # ranges slot per query: as many "cells" as queries)
            assert any(0 < att[l] <= 16384 and cells[l] == att[l] for l in range(1, L)), (att, cells)
