"""Pins of the oracle's grid index (Sec. 3.1) and search-distance selection
(Sec. 4.4) against closed forms, brute-force reformulations and hand-built
examples."""

import itertools
import math

import numpy as np
import pytest

from paper_1810_04758_amd import datagen


def _lattice_id(c, m):
    v = 0
    for x in c:
        v = v * m + x
    return v


@pytest.mark.parametrize("n,m", [(2, 6), (3, 4), (5, 3)])
def test_lattice_unit_cells(oracle_mod, n, m):
    # cell side 1 on the integer lattice: every point is alone in its cell, the
    # key is the row-major lattice id, and the sort is the identity.
    D = datagen.lattice(m, n)
    N = D.shape[0]
    g = oracle_mod.grid(D, 1.0)
    assert (g["lo"] == 0).all() and (g["hi"] == m - 1).all()
    assert g["g"].tolist() == [m] * n
    assert g["keys"].tolist() == list(range(N))
    assert g["perm"].tolist() == list(range(N))
    assert g["cell_keys"].tolist() == list(range(N))
    assert g["cell_start"].tolist() == list(range(N + 1))
    # row segment for offset o (o_0 slowest) of cell c covers the lattice
    # points c + (o, -1..1) that exist
    R = 3 ** (n - 1)
    for cid in range(0, N, max(1, N // 17)):
        c = [int(x) for x in D[cid]]
        for r, o in enumerate(itertools.product((-1, 0, 1), repeat=n - 1)):
            base = [c[j] + o[j] for j in range(n - 1)]
            ids = []
            if all(0 <= b < m for b in base):
                for t in (-1, 0, 1):
                    last = c[-1] + t
                    if 0 <= last < m:
                        ids.append(_lattice_id(base + [last], m))
            s, e = g["ranges"][cid, r]
            if ids:
                assert (s, e) == (min(ids), max(ids) + 1)
            else:
                assert (s, e) == (0, 0)
        assert g["ranges"].shape == (N, R, 2)


def test_lattice_double_cells(oracle_mod):
    # cell side 2 on {0..5}^2: 3x3 cells of 4 points each, keys by floor(x/2)
    D = datagen.lattice(6, 2)
    g = oracle_mod.grid(D, 0.5)
    assert g["g"].tolist() == [3, 3]
    exp_keys = [(int(x) // 2) * 3 + int(y) // 2 for x, y in D]
    assert g["keys"].tolist() == exp_keys
    assert g["cell_keys"].tolist() == list(range(9))
    assert g["cell_start"].tolist() == [4 * k for k in range(10)]


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_grid_matches_bruteforce_membership(oracle_mod, n):
    # Reformulation: a sorted position p belongs to row segment (c, o) iff the
    # cell coordinates of its point equal c's plus o in dims 0..n-2 and lie
    # within one of c's in the last dim.  The oracle's ranges must be exactly
    # the (contiguous) sets of such positions.
    D = datagen.exponential(400, n, seed=30 + n)
    lo, hi = oracle_mod.bounds(D)
    inv_w = 1.0 / 0.05
    g = oracle_mod.grid(D, inv_w)
    coords = np.floor((D - lo) * inv_w).astype(np.int64)
    assert (coords.max(axis=0) + 1 == g["g"]).all()
    # stable sort: keys non-decreasing, ids increasing within a key
    sk, perm = g["sorted_keys"], g["perm"]
    assert (np.diff(sk.astype(np.float64)) >= 0).all()
    same = sk[1:] == sk[:-1]
    assert (perm[1:][same] > perm[:-1][same]).all()
    assert sorted(perm.tolist()) == list(range(D.shape[0]))
    sc = coords[perm]
    ck, cs = g["cell_keys"], g["cell_start"]
    for c in range(ck.shape[0]):
        cc = sc[cs[c]]
        assert (sc[cs[c]:cs[c + 1]] == cc).all()
        for r, o in enumerate(itertools.product((-1, 0, 1), repeat=n - 1)):
            want = np.ones(D.shape[0], dtype=bool)
            for j in range(n - 1):
                want &= sc[:, j] == cc[j] + o[j]
            want &= np.abs(sc[:, n - 1] - cc[n - 1]) <= 1
            pos = np.nonzero(want)[0]
            s, e = g["ranges"][c, r]
            if pos.size:
                assert (s, e) == (pos.min(), pos.max() + 1)
                assert pos.size == e - s
            else:
                assert (s, e) == (0, 0)


def test_grid_dims_product_and_key_range(oracle_mod):
    D = datagen.uniform(3000, 3, seed=4)
    lo, hi = oracle_mod.bounds(D)
    inv_w = 1.0 / 7.5
    gd = oracle_mod.grid_dims(lo, hi, inv_w)
    keys = oracle_mod.cell_keys(D, lo, inv_w, gd)
    assert int(keys.max()) < int(np.prod(gd))
    # decoding the key gives back floor((x - lo) * inv_w)
    coords = np.floor((D - lo) * inv_w).astype(np.int64)
    k = keys.astype(np.int64)
    for j in range(2, -1, -1):
        assert (k % gd[j] == coords[:, j]).all()
        k //= gd[j]


# ---------------------------------------------------------------------------
# Search-distance selection (Sec. 4.4)
# ---------------------------------------------------------------------------

def test_sample_mean_closed_forms(oracle_mod):
    D = np.array([[0.0, 0.0], [3.0, 0.0], [3.0, 4.0], [9.0, 9.0]])
    assert oracle_mod.sample_mean_dist(D, [0, 1, 2]) == 4.0
    sq = datagen.lattice(2, 2)
    m = oracle_mod.sample_mean_dist(sq, [0, 1, 2, 3])
    assert abs(m - (4.0 + 2.0 * math.sqrt(2.0)) / 6.0) < 1e-15


def test_histogram_lattice_closed_form(oracle_mod):
    # sample points on the integer lattice, bin width 1: a distance sqrt(k)
    # (k integer) falls into bin isqrt(k).
    m, n = 9, 2
    D = datagen.lattice(m, n)
    sample = [0, 40, 80, 13]
    n_bins = 7
    counts = oracle_mod.dist_histogram(D, sample, 1.0, n_bins)
    exp = [0] * n_bins
    for s in sample:
        cs = D[s].astype(int)
        for j in range(D.shape[0]):
            if j == s:
                continue
            k = int(((D[j].astype(int) - cs) ** 2).sum())
            b = math.isqrt(k)
            if b < n_bins:
                exp[b] += 1
    assert counts.tolist() == exp


def test_histogram_duplicates_and_bounds(oracle_mod):
    # duplicates of a sample point land in bin 0; the self pair is skipped;
    # distances at or beyond n_bins * width are not stored
    D = np.array([[0.0], [0.0], [0.5], [1.0], [2.0]])
    counts = oracle_mod.dist_histogram(D, [0], 2.0, 4)  # width 0.5
    assert counts.tolist() == [1, 1, 1, 0]


def test_eps_min_rule(oracle_mod):
    counts = [0, 2, 3, 5]
    bw = 0.5
    # cumulative 0, 2, 5, 10
    assert oracle_mod.eps_min(counts, bw, 1, 4) == 1.25
    assert oracle_mod.eps_min(counts, bw, 2, 2) == 1.25
    assert oracle_mod.eps_min(counts, bw, 1, 2) == 0.75
    assert oracle_mod.eps_min(counts, bw, 1, 6) == 1.75
    assert oracle_mod.eps_min(counts, bw, 1, 11) == 2.0


def test_eps_min_uniform_density_statistical(oracle_mod):
    # parity unpinned (random sample): on uniform 2-D data the ball of radius
    # eps_min holds about K points, i.e. pi eps^2 rho ~ K (edge effects lower
    # the histogram count, so eps_min comes out slightly large).
    N, K = 40000, 16
    D = datagen.uniform(N, 2, seed=3)
    s_mean = datagen.sample_ids(N, 40, seed=9)
    eps_mean = oracle_mod.sample_mean_dist(D, s_mean)
    n_bins = 1000
    sample = datagen.sample_ids(N, 50, seed=10)
    counts = oracle_mod.dist_histogram(D, sample, n_bins / eps_mean, n_bins)
    e = oracle_mod.eps_min(counts, eps_mean / n_bins, len(sample), K)
    rho = N / 100.0 ** 2
    e_closed = math.sqrt(K / (math.pi * rho))
    assert 0.85 * e_closed < e < 1.25 * e_closed


def test_splitmix64_published_outputs(oracle_mod):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           "splitmix64_seed0.json")) as f:
        g = json.load(f)
    got = [int(v) for v in oracle_mod.splitmix64(g["seed"], len(g["outputs_hex"]))]
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_sample_ids_draws_distinct_residues(oracle_mod):
    # without replacement: the first `count` distinct generator residues mod N,
    # increasing; every id when count >= N
    N, count, seed = 1000, 300, 12345
    ids = oracle_mod.sample_ids(N, count, seed)
    assert ids.shape == (count,) and (np.diff(ids) > 0).all() and ids[0] >= 0 and ids[-1] < N
    stream = oracle_mod.splitmix64(seed, 5000) % np.uint64(N)
    _, first = np.unique(stream, return_index=True)
    expect = np.sort(stream[np.sort(first)][:count].astype(np.int64))
    assert (ids == expect).all()
    assert (oracle_mod.sample_ids(7, 50, 3) == np.arange(7)).all()
