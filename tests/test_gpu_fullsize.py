"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times (default options, device inputs and outputs).

Every row of every workload is compared with the oracle: ids identical and
distances bit-identical.  At these sizes the oracle answers through its exact
kd-tree search (one search at the largest K of a dataset; the K nearest in
(d^2, id) order are a prefix of the larger K's list).  That search is itself
checked against the brute-force definition on the rows that matter most at
full size: random rows, the sparsest rows (largest K-th distance: the ones
that reach the late grid levels and the brute-force tail) and the densest
rows (smallest K-th distance: the crowded cells of the heavy-query path).
Each test prints how many rows each level, the heavy-query kernel and the
tail solved: every one of them was checked.
"""

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


def _paths(st):
    """Rows solved by each path of one join (from the join's statistics)."""
    out = []
    for L in range(st["levels"]):
        solved = st["attempted"][L] - st["failed"][L]
        heavy = st["heavy_queries"][L] - st["heavy_failed"][L]
        out.append(f"L{L}:{solved}(heavy {heavy})")
    out.append(f"tail:{st['tail_queries']}")
    return " ".join(out)


@pytest.mark.parametrize("name,Ks", WORKLOADS, ids=[w[0] for w in WORKLOADS])
def test_fullsize_every_row(api, oracle_mod, name, Ks):
    import torch
    D, _, _ = datagen.config_points(name)
    N = D.shape[0]
    Kmax = max(Ks)
    print(f"[fullsize] {name} N={N} K={Ks}", flush=True)
    ref_ids, ref_d = oracle_mod.knn_kdtree(D, Kmax)

    # the kd-tree search against the definition on random, sparsest and
    # densest rows (chosen from the oracle's own K-th distances)
    rng = np.random.default_rng(123)
    kth = ref_d[:, Kmax - 1]
    order = np.argsort(kth, kind="stable")
    nsel = 64 if N > 10_000_000 else 256
    rows = np.unique(np.concatenate([rng.choice(N, size=nsel, replace=False), order[-nsel:],
                                     order[:nsel], [0, N - 1]]))
    bf_ids, bf_d = oracle_mod.knn(D, Kmax, rows=rows)
    assert (bf_ids == ref_ids[rows]).all() and (bf_d == ref_d[rows]).all(), \
        "kd-tree oracle differs from the brute-force definition"

    Dd = torch.from_numpy(D).cuda()
    idx = api.build_index(Dd)
    for K in Ks:
        ids, dists, st = idx.self_join(K, with_stats=True)
        torch.cuda.synchronize()
        print(f"  K={K} levels={st['levels']} ms={st['ms_total']:.1f} rows per path: "
              f"{_paths(st)}", flush=True)
        got_i = ids.cpu().numpy()
        got_d = dists.cpu().numpy()
        del ids, dists
        bad = np.nonzero((got_i != ref_ids[:, :K]).any(axis=1) |
                         (got_d != ref_d[:, :K]).any(axis=1))[0]
        assert bad.size == 0, f"{bad.size} of {N} rows differ, e.g. row {bad[0]}"
    idx.close()
    del Dd
    torch.cuda.empty_cache()
