"""CPU oracle for the grid KNN self-join (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``liboracle.so`` built from
``knn_oracle.cpp`` (plain C++, fp64, no contraction) and shares nothing with
the HIP library.  Each wrapper names the passage of the paper it follows.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC]


def build():
    """Compile liboracle.so (always recompiles)."""
    subprocess.check_call(BUILD_CMD)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_knn.argtypes = [P, i64, i32, i32, P, i64, P, P, i32]
        L.oracle_knn.restype = ctypes.c_int
        L.oracle_knn_kdtree.argtypes = [P, i64, i32, i32, P, i64, P, P, i32]
        L.oracle_knn_kdtree.restype = ctypes.c_int
        L.oracle_knn_rs.argtypes = [P, i64, P, i64, i32, i32, P, i64, P, P, i32]
        L.oracle_knn_rs.restype = ctypes.c_int
        L.oracle_eps_join.argtypes = [P, i64, i32, f64, P, i64, P, P, P, P, i32]
        L.oracle_eps_join.restype = ctypes.c_int
        L.oracle_sq_dist.argtypes = [P, i32, i64, i64]
        L.oracle_sq_dist.restype = f64
        L.oracle_bounds.argtypes = [P, i64, i32, P, P]
        L.oracle_grid_dims.argtypes = [P, P, i32, f64, P]
        L.oracle_cell_keys.argtypes = [P, i64, i32, P, f64, P, P]
        L.oracle_grid_build.argtypes = [P, i64, P, P, P, P]
        L.oracle_grid_build.restype = i64
        L.oracle_neighbor_ranges.argtypes = [P, P, i64, i32, P, P]
        L.oracle_sample_mean_dist.argtypes = [P, i32, P, i64]
        L.oracle_sample_mean_dist.restype = f64
        L.oracle_dist_histogram.argtypes = [P, i64, i32, P, i64, f64, i32, P]
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64, i64, P]
        L.oracle_sample_ids.argtypes = [i64, i64, ctypes.c_uint64, P]
        L.oracle_eps_min.argtypes = [P, i32, f64, i64, i32]
        L.oracle_eps_min.restype = f64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(D):
    D = np.ascontiguousarray(D, dtype=np.float64)
    if D.ndim != 2:
        raise ValueError("D must be N x n")
    return D


def knn(D, K, rows=None, threads=0):
    """K nearest neighbours of the given rows by the definition (Sec. 2.1).

    Returns (ids int32 [nrows, K], dists float64 [nrows, K]); ties in the squared
    distance go to the lower id, the point itself is excluded by id.
    """
    D = _f64(D)
    N, n = D.shape
    if rows is None:
        nrows = N
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows.shape[0]
        rp = _p(rows)
    ids = np.empty((nrows, K), dtype=np.int32)
    dists = np.empty((nrows, K), dtype=np.float64)
    rc = lib().oracle_knn(_p(D), N, n, K, rp, nrows, _p(ids), _p(dists), threads)
    if rc != 0:
        raise ValueError("oracle_knn: invalid arguments")
    return ids, dists


def knn_kdtree(D, K, rows=None, threads=0):
    """The same result as knn() (Sec. 2.1 definition) through an exact kd-tree
    search, for sizes where brute force is too slow.  Pinned to knn() by the
    tests; same arguments and outputs."""
    D = _f64(D)
    N, n = D.shape
    if rows is None:
        nrows = N
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows.shape[0]
        rp = _p(rows)
    ids = np.empty((nrows, K), dtype=np.int32)
    dists = np.empty((nrows, K), dtype=np.float64)
    rc = lib().oracle_knn_kdtree(_p(D), N, n, K, rp, nrows, _p(ids), _p(dists), threads)
    if rc != 0:
        raise ValueError("oracle_knn_kdtree: invalid arguments")
    return ids, dists


def knn_rs(S, Q, K, rows=None, threads=0):
    """KNN join of two sets (Sec. 2.1, R join S): for each row of Q (or the
    given rows of Q) its K nearest points of S by (d^2, S id), nothing
    excluded.  Returns (ids int32 [nrows, K] of S, dists float64)."""
    S = _f64(S)
    Q = _f64(Q)
    if S.shape[1] != Q.shape[1]:
        raise ValueError("S and Q must have the same dimension")
    NQ, n = Q.shape
    if rows is None:
        nrows = NQ
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows.shape[0]
        rp = _p(rows)
    ids = np.empty((nrows, K), dtype=np.int32)
    dists = np.empty((nrows, K), dtype=np.float64)
    rc = lib().oracle_knn_rs(_p(S), S.shape[0], _p(Q), NQ, n, K, rp, nrows, _p(ids), _p(dists),
                             threads)
    if rc != 0:
        raise ValueError("oracle_knn_rs: invalid arguments")
    return ids, dists


def eps_join(D, eps, rows=None, threads=0):
    """Distance similarity self-join (the range-query join the paper builds
    on): every pair (i, j), j != i, with dist(i, j) <= eps, for every point
    i (or the given rows), grouped by row in row order, j ascending.
    Returns (q int32, j int32, dist float64, counts int64 per row)."""
    D = _f64(D)
    N, n = D.shape
    if rows is None:
        nrows = N
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows.shape[0]
        rp = _p(rows)
    counts = np.empty(nrows, dtype=np.int64)
    L = lib()
    if L.oracle_eps_join(_p(D), N, n, float(eps), rp, nrows, _p(counts), None, None, None,
                         threads) != 0:
        raise ValueError("oracle_eps_join: invalid arguments")
    tot = int(counts.sum())
    q = np.empty(tot, dtype=np.int32)
    j = np.empty(tot, dtype=np.int32)
    d = np.empty(tot, dtype=np.float64)
    if L.oracle_eps_join(_p(D), N, n, float(eps), rp, nrows, _p(counts), _p(q), _p(j), _p(d),
                         threads) != 0:
        raise ValueError("oracle_eps_join: invalid arguments")
    return q, j, d, counts


def sq_dist(D, a, b):
    D = _f64(D)
    return lib().oracle_sq_dist(_p(D), D.shape[1], a, b)


def bounds(D):
    D = _f64(D)
    n = D.shape[1]
    lo = np.empty(n)
    hi = np.empty(n)
    lib().oracle_bounds(_p(D), D.shape[0], n, _p(lo), _p(hi))
    return lo, hi


def grid_dims(lo, hi, inv_w):
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    g = np.empty(lo.shape[0], dtype=np.int64)
    lib().oracle_grid_dims(_p(lo), _p(hi), lo.shape[0], inv_w, _p(g))
    return g


def cell_keys(D, lo, inv_w, g):
    D = _f64(D)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.int64)
    keys = np.empty(D.shape[0], dtype=np.uint64)
    lib().oracle_cell_keys(_p(D), D.shape[0], D.shape[1], _p(lo), inv_w, _p(g), _p(keys))
    return keys


def grid_build(keys):
    """Stable sort by cell key and the non-empty cell table (Sec. 3.1)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    N = keys.shape[0]
    sk = np.empty(N, dtype=np.uint64)
    perm = np.empty(N, dtype=np.int32)
    ck = np.empty(N, dtype=np.uint64)
    cs = np.empty(N + 1, dtype=np.int64)
    M = lib().oracle_grid_build(_p(keys), N, _p(sk), _p(perm), _p(ck), _p(cs))
    return sk, perm, ck[:M].copy(), cs[:M + 1].copy()


def neighbor_ranges(cell_keys_, cell_start, n, g):
    """Row-segment point ranges of the 3^n adjacent cells of every cell."""
    ck = np.ascontiguousarray(cell_keys_, dtype=np.uint64)
    cs = np.ascontiguousarray(cell_start, dtype=np.int64)
    g = np.ascontiguousarray(g, dtype=np.int64)
    M = ck.shape[0]
    R = 3 ** (n - 1)
    out = np.empty((M, R, 2), dtype=np.int64)
    lib().oracle_neighbor_ranges(_p(ck), _p(cs), M, n, _p(g), _p(out))
    return out


def grid(D, inv_w):
    """Whole grid index at cell width 1/inv_w: dict of every array."""
    lo, hi = bounds(D)
    g = grid_dims(lo, hi, inv_w)
    keys = cell_keys(D, lo, inv_w, g)
    sk, perm, ck, cs = grid_build(keys)
    rng = neighbor_ranges(ck, cs, D.shape[1], g)
    return dict(lo=lo, hi=hi, g=g, keys=keys, sorted_keys=sk, perm=perm,
                cell_keys=ck, cell_start=cs, ranges=rng)


def sample_mean_dist(D, sample):
    """eps_mean of Sec. 4.4: mean distance over pairs inside the sample."""
    D = _f64(D)
    s = np.ascontiguousarray(sample, dtype=np.int64)
    return lib().oracle_sample_mean_dist(_p(D), D.shape[1], _p(s), s.shape[0])


def dist_histogram(D, sample, inv_bin_width, n_bins):
    """Distance histogram of Sec. 4.4 (sample points against all of D)."""
    D = _f64(D)
    s = np.ascontiguousarray(sample, dtype=np.int64)
    counts = np.empty(n_bins, dtype=np.uint64)
    lib().oracle_dist_histogram(_p(D), D.shape[0], D.shape[1], _p(s), s.shape[0],
                                inv_bin_width, n_bins, _p(counts))
    return counts


def splitmix64(seed, count):
    """The first `count` outputs of SplitMix64 from state `seed` (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    lib().oracle_splitmix64(seed & (2 ** 64 - 1), count, _p(out))
    return out


def sample_ids(N, count, seed):
    """Sec. 4.4 sampling: `count` distinct point ids drawn with SplitMix64
    (outputs modulo N, repeats skipped), increasing; every id if count >= N."""
    n = min(count, N)
    out = np.empty(n, dtype=np.int64)
    lib().oracle_sample_ids(N, count, seed & (2 ** 64 - 1), _p(out))
    return out


def eps_min(counts, bin_width, n_sample, K):
    """eps_min of Sec. 4.4 from a cumulative distance histogram."""
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    return lib().oracle_eps_min(_p(c), c.shape[0], bin_width, n_sample, K)
