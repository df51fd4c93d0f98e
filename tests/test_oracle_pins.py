"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formula: expected values come from the
paper's worked figures (hand-derived, stored under tests/golden/), from exact
rational/integer arithmetic on inputs where fp64 is exact, from integer
lattice closed forms, from invariants and from metamorphic relations.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1810_04758_amd import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Worked examples of the paper's figures
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("panel", ["a", "b"])
def test_fig_eps_expansion(oracle_mod, panel):
    g = _load("fig_eps_expansion.json")
    p = g["panels"][panel]
    D = np.array(p["points"], dtype=np.float64)
    K = g["K"]
    ids, dists = oracle_mod.knn(D, K, rows=[0])
    assert ids[0].tolist() == p["knn_ids_of_query"]
    for k, s in enumerate(p["exact_sq_dists"]):
        assert abs(dists[0, k] - math.sqrt(float(Fraction(s)))) <= 1e-15
    # caption facts: how many neighbours each drawn ring holds
    q = D[0]
    d_all = np.sqrt(((D[1:] - q) ** 2).sum(axis=1))
    for label, count in p["count_within_label_radius"].items():
        radius = 0.5 * float(label)
        assert int((d_all <= radius + 1e-12).sum()) == count


def test_fig_eps_expansion_sixth_neighbour_rounding(oracle_mod):
    # Panel (a): the sixth neighbour (0.3, 1.1) is at exact squared distance
    # 1/2, but fp64 (0.3-1)^2 + (1.1-1)^2 rounds below it.
    g = _load("fig_eps_expansion.json")
    D = np.array(g["panels"]["a"]["points"], dtype=np.float64)
    assert oracle_mod.sq_dist(D, 0, 1) == float.fromhex("0x1.fffffffffffffp-2")
    ids, _ = oracle_mod.knn(D, 6, rows=[0])
    assert ids[0, 5] == 1


def test_fig_work_example(oracle_mod):
    g = _load("fig_work_example.json")
    D = np.array(g["points"], dtype=np.float64)
    ids, dists = oracle_mod.knn(D, g["K"] + 1, rows=[0])
    assert ids[0, :3].tolist() == g["knn_ids_of_query"]
    assert ids[0, 3] == g["fourth_neighbour"]["id"]
    for k, s in enumerate(g["exact_sq_dists"]):
        assert abs(dists[0, k] - math.sqrt(float(Fraction(s)))) <= 1e-15


def test_fig_work_example_duplicates_tie_to_lower_id(oracle_mod):
    g = _load("fig_work_example.json")
    D = np.array(g["points"], dtype=np.float64)
    a, b = g["duplicate_pair"]
    N = D.shape[0]
    ids, dists = oracle_mod.knn(D, N - 1)
    # the two copies are each other's nearest neighbour at distance 0
    assert ids[a, 0] == b and dists[a, 0] == 0.0
    assert ids[b, 0] == a and dists[b, 0] == 0.0
    # every other row sees the copies at the same distance, lower id first
    for i in range(N):
        if i in (a, b):
            continue
        row = ids[i].tolist()
        pa, pb = row.index(a), row.index(b)
        assert pb == pa + 1
        assert dists[i, pa] == dists[i, pb]


# ---------------------------------------------------------------------------
# Exact brute force on tiny dyadic inputs (fp64 is exact there)
# ---------------------------------------------------------------------------

def _exact_knn(D, K, bits):
    scale = 2 ** bits
    Z = np.rint(D * scale).astype(np.int64)
    N = Z.shape[0]
    out = []
    for i in range(N):
        cand = []
        for j in range(N):
            if j == i:
                continue
            d2 = int(((Z[i] - Z[j]) ** 2).sum())
            cand.append((d2, j))
        cand.sort()
        out.append(cand[:K])
    return out, scale * scale


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_exact_bruteforce_dyadic(oracle_mod, n):
    D = datagen.dyadic(120, n, seed=100 + n, bits=3, span=2)  # many exact ties
    N = D.shape[0]
    for K in (1, 7, N - 1):
        ids, dists = oracle_mod.knn(D, K)
        exact, s2 = _exact_knn(D, K, bits=3)
        for i in range(N):
            assert ids[i].tolist() == [j for _, j in exact[i]]
            for k, (d2, _) in enumerate(exact[i]):
                assert dists[i, k] == math.sqrt(d2 / s2)


# ---------------------------------------------------------------------------
# Integer lattice closed forms
# ---------------------------------------------------------------------------

def _lattice_id(c, m):
    v = 0
    for x in c:
        v = v * m + x
    return v


def _lattice_expected(c, m, n, rmax):
    import itertools
    out = []
    for o in itertools.product(range(-rmax, rmax + 1), repeat=n):
        if all(x == 0 for x in o):
            continue
        p = [c[j] + o[j] for j in range(n)]
        if min(p) < 0 or max(p) >= m:
            continue
        out.append((sum(x * x for x in o), _lattice_id(p, m)))
    out.sort()
    # keep the prefix whose squared distance is certainly complete (<= rmax^2)
    return [e for e in out if e[0] <= rmax * rmax]


@pytest.mark.parametrize("n,m", [(2, 9), (3, 7), (4, 6), (6, 5)])
def test_lattice_interior_and_corner(oracle_mod, n, m):
    D = datagen.lattice(m, n)
    center = [m // 2] * n
    corner = [0] * n
    rows = [_lattice_id(center, m), _lattice_id(corner, m)]
    rmax = 2
    for row, c in zip(rows, (center, corner)):
        exp = _lattice_expected(c, m, n, rmax)
        K = len(exp)
        ids, dists = oracle_mod.knn(D, K, rows=[row])
        assert ids[0].tolist() == [j for _, j in exp]
        assert dists[0].tolist() == [math.sqrt(d2) for d2, _ in exp]
    # closed form counts: an interior point has 2n neighbours at distance 1,
    # then 2n(n-1) at sqrt(2); a corner has n at distance 1
    ids, dists = oracle_mod.knn(D, 2 * n + 2 * n * (n - 1), rows=rows[:1])
    assert (dists[0, :2 * n] == 1.0).all()
    assert (dists[0, 2 * n:] == math.sqrt(2.0)).all()
    ids, dists = oracle_mod.knn(D, n, rows=rows[1:])
    assert sorted(ids[0].tolist()) == sorted(m ** (n - 1 - j) for j in range(n))
    assert (dists[0] == 1.0).all()


# ---------------------------------------------------------------------------
# Invariants and metamorphic relations on continuous random data
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 4, 6])
def test_invariants(oracle_mod, n):
    D = datagen.uniform(1500, n, seed=7 + n)
    N = D.shape[0]
    K = 17
    ids, dists = oracle_mod.knn(D, K)
    for i in range(0, N, 37):
        row = ids[i].tolist()
        assert len(set(row)) == K and i not in row
        d2 = [oracle_mod.sq_dist(D, i, j) for j in row]
        assert all((d2[k], row[k]) < (d2[k + 1], row[k + 1]) for k in range(K - 1))
        assert dists[i].tolist() == [math.sqrt(x) for x in d2]
        # completeness: nothing outside the list precedes the K-th entry
        last = (d2[-1], row[-1])
        outside = [j for j in range(N) if j != i and j not in row]
        assert all((oracle_mod.sq_dist(D, i, j), j) > last for j in outside)


def test_scale_by_power_of_two(oracle_mod):
    D = datagen.uniform(800, 3, seed=11)
    ids, dists = oracle_mod.knn(D, 9)
    ids2, dists2 = oracle_mod.knn(D * 8.0, 9)
    assert (ids == ids2).all()
    assert (dists2 == dists * 8.0).all()


def test_relabel_permutes_ids(oracle_mod):
    D = datagen.uniform(700, 2, seed=12)
    ids, dists = oracle_mod.knn(D, 6)
    rng = np.random.default_rng(5)
    p = rng.permutation(D.shape[0])      # new row r holds old point p[r]
    inv = np.empty_like(p)
    inv[p] = np.arange(p.shape[0])
    ids2, dists2 = oracle_mod.knn(D[p], 6)
    assert (inv[ids[p]] == ids2).all()
    assert (dists[p] == dists2).all()


def test_rows_subset_matches_full(oracle_mod):
    D = datagen.exponential(600, 4, seed=13)
    ids, dists = oracle_mod.knn(D, 5)
    rows = np.array([0, 599, 17, 17, 300])
    ids2, dists2 = oracle_mod.knn(D, 5, rows=rows)
    assert (ids[rows] == ids2).all() and (dists[rows] == dists2).all()


def test_invalid_k(oracle_mod):
    D = datagen.uniform(10, 2, seed=1)
    with pytest.raises(ValueError):
        oracle_mod.knn(D, 10)
    with pytest.raises(ValueError):
        oracle_mod.knn(D, 0)
    ids, _ = oracle_mod.knn(D, 9)
    assert sorted(ids[0].tolist()) == list(range(1, 10))
