"""Pins of the oracle's kd-tree search (oracle.knn_kdtree), the exact KNN of
the Sec. 2.1 definition answered with pruning so that the benchmark
workloads can be checked on every row.

It is pinned to the brute-force definition (oracle.knn, itself pinned by
test_oracle_pins.py) on many distributions, and directly to exact integer
arithmetic where fp64 is exact (dyadic inputs with many exact ties, integer
lattices), so that a wrong prune (a lost tie, a skipped box, the point
itself kept) fails here.
"""

import math

import numpy as np
import pytest

from paper_1810_04758_amd import datagen


def _same(a, b):
    return bool((a[0] == b[0]).all() and (a[1] == b[1]).all())


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_kdtree_equals_definition_uniform(oracle_mod, n):
    D = datagen.uniform(3000, n, seed=200 + n)
    for K in (1, 8, 33):
        assert _same(oracle_mod.knn_kdtree(D, K), oracle_mod.knn(D, K))


@pytest.mark.parametrize("n", [2, 4, 6])
def test_kdtree_equals_definition_exponential(oracle_mod, n):
    D = datagen.exponential(4000, n, seed=210 + n)
    for K in (1, 16, 64):
        assert _same(oracle_mod.knn_kdtree(D, K), oracle_mod.knn(D, K))


def test_kdtree_equals_definition_clustered(oracle_mod):
    # tight clusters (sigma down to 1e-3) beside a sparse background
    D = datagen.clustered(12000, seed=220, n_clusters=40, sigma_lo=1e-3, sigma_hi=2.0)
    for K in (1, 16, 100):
        assert _same(oracle_mod.knn_kdtree(D, K), oracle_mod.knn(D, K))


@pytest.mark.parametrize("n", [2, 3, 6])
def test_kdtree_exact_ties_dyadic(oracle_mod, n):
    # coordinates in {0, 1/2, 1, 3/2}: hundreds of exact duplicates and ties;
    # expected lists by exact integer arithmetic, ties to the lower id
    D = datagen.dyadic(400, n, seed=230 + n, bits=1, span=2)
    Z = np.rint(D * 2).astype(np.int64)
    N = D.shape[0]
    for K in (5, 60, N - 1):
        ids, dists = oracle_mod.knn_kdtree(D, K)
        for i in range(0, N, 7):
            d2 = ((Z - Z[i]) ** 2).sum(axis=1)
            cand = sorted((int(d2[j]), j) for j in range(N) if j != i)[:K]
            assert ids[i].tolist() == [j for _, j in cand]
            assert dists[i].tolist() == [math.sqrt(v / 4.0) for v, _ in cand]


@pytest.mark.parametrize("n,m", [(2, 30), (3, 9), (4, 6)])
def test_kdtree_lattice_shells(oracle_mod, n, m):
    # every point of the lattice: its 2n neighbours at distance 1 then 2n(n-1)
    # at sqrt(2) where the lattice has them; kd split planes fall on lattice
    # coordinates, so ties sit exactly on box faces
    D = datagen.lattice(m, n)
    K = 2 * n
    ids, dists = oracle_mod.knn_kdtree(D, K)
    ref = oracle_mod.knn(D, K)
    assert _same((ids, dists), ref)
    interior = np.all((D > 0) & (D < m - 1), axis=1)
    assert (dists[interior] == 1.0).all()


def test_kdtree_all_identical_and_two_points(oracle_mod):
    D = np.full((50, 3), 2.5)
    ids, dists = oracle_mod.knn_kdtree(D, 49)
    assert (dists == 0).all()
    for i in range(50):
        assert ids[i].tolist() == [j for j in range(50) if j != i]
    ids, dists = oracle_mod.knn_kdtree(np.array([[0.0, 0.0], [3.0, 4.0]]), 1)
    assert ids.tolist() == [[1], [0]] and dists.tolist() == [[5.0], [5.0]]


@pytest.mark.parametrize("scale", [2.0 ** -70, 2.0 ** 60])
def test_kdtree_scale_by_power_of_two(oracle_mod, scale):
    D = datagen.exponential(3000, 3, seed=240)
    ids, dists = oracle_mod.knn_kdtree(D, 12)
    ids2, dists2 = oracle_mod.knn_kdtree(D * scale, 12)
    assert (ids == ids2).all() and (dists2 == dists * scale).all()


def test_kdtree_rows_subset_and_invalid(oracle_mod):
    D = datagen.uniform(2000, 4, seed=250)
    full = oracle_mod.knn_kdtree(D, 9)
    rows = np.array([1999, 0, 5, 5, 1000])
    sub = oracle_mod.knn_kdtree(D, 9, rows=rows)
    assert (full[0][rows] == sub[0]).all() and (full[1][rows] == sub[1]).all()
    with pytest.raises(ValueError):
        oracle_mod.knn_kdtree(D, 2000)
    with pytest.raises(ValueError):
        oracle_mod.knn_kdtree(D, 3, rows=np.array([2000]))
