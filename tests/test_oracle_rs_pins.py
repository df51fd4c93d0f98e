"""Pins of the oracle's KNN join of two sets, R join_KNN S (Sec. 2.1: the
self-join's definition applied to a query set R and a searched set S, nothing
excluded), against facts that do not come from the oracle's own formula:
exact integer brute force on dyadic inputs (queries inside and far outside
S's bounding box), the relation to the pinned self-join (R = S: every point's
own copy comes first unless a lower-id duplicate shares distance 0, and the
rest is the self-join's row), the paper's figure with its query point taken
out of the set, and metamorphic relations."""

import json
import math
import os

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _exact_rs(S, Q, K, bits):
    scale = 2 ** bits
    ZS = np.rint(S * scale).astype(np.int64)
    ZQ = np.rint(Q * scale).astype(np.int64)
    out = []
    for q in ZQ:
        cand = sorted((int(((q - s) ** 2).sum()), j) for j, s in enumerate(ZS))
        out.append(cand[:K])
    return out, scale * scale


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_exact_bruteforce_dyadic(oracle_mod, n):
    S = datagen.dyadic(150, n, seed=200 + n, bits=3, span=2)   # many exact ties
    Q = datagen.dyadic(40, n, seed=300 + n, bits=3, span=3)    # some outside S's box
    Q = np.concatenate([Q, S[:5], np.full((1, n), 40.0)])       # copies of S points, a far one
    for K in (1, 9, S.shape[0]):
        ids, dists = oracle_mod.knn_rs(S, Q, K)
        exact, s2 = _exact_rs(S, Q, K, bits=3)
        for r in range(Q.shape[0]):
            assert ids[r].tolist() == [j for _, j in exact[r]]
            assert dists[r].tolist() == [math.sqrt(d2 / s2) for d2, _ in exact[r]]


def test_self_relation(oracle_mod):
    # R = S: row i of R join S holds i itself at distance 0, behind any
    # lower-id duplicate; without it, the row is the self-join's
    base = datagen.dyadic(120, 3, seed=7, bits=2, span=2)
    D = np.concatenate([base, base[:15]])  # exact duplicates
    N = D.shape[0]
    K = 8
    ids, dists = oracle_mod.knn_rs(D, D, K + 1)
    ref_i, ref_d = oracle_mod.knn(D, K)
    for i in range(N):
        row = ids[i].tolist()
        assert i in row and dists[i, row.index(i)] == 0.0
        assert all(dists[i, k] == 0.0 and D[row[k]].tolist() == D[i].tolist()
                   for k in range(row.index(i)))
        rest = [j for j in row if j != i][:K]
        assert rest == ref_i[i].tolist()


@pytest.mark.parametrize("panel", ["a", "b"])
def test_figure_query_outside_the_set(oracle_mod, panel):
    # the figure's query point (id 0) answered against the other points only
    with open(os.path.join(GOLDEN, "fig_eps_expansion.json")) as f:
        g = json.load(f)
    p = g["panels"][panel]
    D = np.array(p["points"], dtype=np.float64)
    ids, _ = oracle_mod.knn_rs(D[1:], D[:1], g["K"])
    assert (ids[0] + 1).tolist() == p["knn_ids_of_query"]


def test_metamorphic(oracle_mod):
    S = datagen.uniform(900, 4, seed=21)
    Q = datagen.uniform(300, 4, seed=22)
    ids, dists = oracle_mod.knn_rs(S, Q, 7)
    rng = np.random.default_rng(3)
    pq = rng.permutation(Q.shape[0])
    i2, d2 = oracle_mod.knn_rs(S, Q[pq], 7)
    assert (i2 == ids[pq]).all() and (d2 == dists[pq]).all()
    ps = rng.permutation(S.shape[0])   # new S row r holds old point ps[r]
    inv = np.empty_like(ps)
    inv[ps] = np.arange(ps.shape[0])
    i3, d3 = oracle_mod.knn_rs(S[ps], Q, 7)
    assert (inv[ids] == i3).all() and (d3 == dists).all()
    i4, d4 = oracle_mod.knn_rs(S * 4.0, Q * 4.0, 7)
    assert (i4 == ids).all() and (d4 == dists * 4.0).all()
    rows = np.array([5, 0, 299, 5])
    i5, d5 = oracle_mod.knn_rs(S, Q, 7, rows=rows)
    assert (i5 == ids[rows]).all() and (d5 == dists[rows]).all()


def test_invalid(oracle_mod):
    S = datagen.uniform(10, 2, seed=1)
    Q = datagen.uniform(3, 2, seed=2)
    with pytest.raises(ValueError):
        oracle_mod.knn_rs(S, Q, 11)
    with pytest.raises(ValueError):
        oracle_mod.knn_rs(S, Q, 0)
    with pytest.raises(ValueError):
        oracle_mod.knn_rs(S, datagen.uniform(3, 3, seed=2), 2)
    ids, _ = oracle_mod.knn_rs(S, Q, 10)
    assert all(sorted(r) == list(range(10)) for r in ids.tolist())
