"""Seeded synthetic point sets shaped like the paper's workloads.

This module only draws random numbers (numpy PCG64); it holds none of the
method's arithmetic, so the HIP path and the CPU oracle can both be fed from
it.  Shapes and distributions follow the paper's experimental datasets
(Sec. 5.1): uniformly distributed points, exponentially distributed points
with rate 40, and a two-dimensional catalogue-like set standing in for the
real-world astronomy positions, which are not available here.
"""

import numpy as np


def uniform(N, n, seed, lo=0.0, hi=100.0):
    """N points i.i.d. uniform in [lo, hi)^n (the Unif-nD shape)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(N, n))


def exponential(N, n, seed, rate=40.0):
    """N points, every coordinate i.i.d. exponential with the given rate
    (the Expo-nD shape: a dense corner and a sparse tail)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.exponential(1.0 / rate, size=(N, n))


def clustered(N, seed, n_clusters=500, frac_clustered=0.7,
              sigma_lo=0.05, sigma_hi=2.0):
    """2-D catalogue-shaped points: a fraction drawn from isotropic Gaussian
    clusters (centres uniform in [0,360) x [-90,90), sigma log-uniform in
    [sigma_lo, sigma_hi]), the rest uniform on the same box; shuffled."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_cl = int(round(N * frac_clustered))
    n_bg = N - n_cl
    cx = rng.uniform(0.0, 360.0, size=n_clusters)
    cy = rng.uniform(-90.0, 90.0, size=n_clusters)
    sig = np.exp(rng.uniform(np.log(sigma_lo), np.log(sigma_hi), size=n_clusters))
    which = rng.integers(0, n_clusters, size=n_cl)
    pts_cl = np.empty((n_cl, 2))
    pts_cl[:, 0] = cx[which] + sig[which] * rng.standard_normal(n_cl)
    pts_cl[:, 1] = cy[which] + sig[which] * rng.standard_normal(n_cl)
    pts_bg = np.empty((n_bg, 2))
    pts_bg[:, 0] = rng.uniform(0.0, 360.0, size=n_bg)
    pts_bg[:, 1] = rng.uniform(-90.0, 90.0, size=n_bg)
    pts = np.concatenate([pts_cl, pts_bg], axis=0)
    rng.shuffle(pts, axis=0)
    return pts


def dyadic(N, n, seed, bits=6, span=8):
    """Points whose coordinates are multiples of 2^-bits in [0, span): every
    squared distance between them is exact in fp64, so exact rational
    arithmetic gives the same order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = 2 ** bits
    return rng.integers(0, span * scale, size=(N, n)).astype(np.float64) / scale


def lattice(m, n):
    """All points of the integer lattice {0..m-1}^n, in row-major order (the
    last coordinate varies fastest)."""
    axes = [np.arange(m, dtype=np.float64)] * n
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.reshape(-1) for a in mesh], axis=1)


def sample_ids(N, count, seed):
    """count distinct point ids drawn without replacement (sorted)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, N)
    return np.sort(rng.choice(N, size=count, replace=False)).astype(np.int64)


def serving_pool(count=24, seed=6, n_lo=1e4, n_hi=1e7):
    """Resident datasets of the serving workload: N log-uniform in [n_lo, n_hi],
    dims uniform in {2,3,4,6}, coordinates uniform [0,100) or exponential(40)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        N = int(round(10 ** rng.uniform(np.log10(n_lo), np.log10(n_hi))))
        n = int(rng.choice([2, 3, 4, 6]))
        if rng.uniform() < 0.5:
            D = uniform(N, n, seed=seed * 1000 + i)
            kind = "uniform"
        else:
            D = exponential(N, n, seed=seed * 1000 + i)
            kind = "exponential"
        out.append((D, f"{kind} {n}-D N={N}"))
    return out


def serving_trace(seconds, rate, n_datasets, seed=7, Ks=(1, 4, 16, 64)):
    """Poisson arrivals (mean `rate` per second) over `seconds`: arrival
    times, dataset indexes (uniform) and K values (uniform over Ks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.cumsum(rng.exponential(1.0 / rate, size=int(seconds * rate * 2) + 16))
    t = t[t < seconds]
    ds = rng.integers(0, n_datasets, size=t.shape[0])
    ks = rng.choice(np.array(Ks), size=t.shape[0])
    return t, ds, ks


# Workloads of the benchmark configurations (seeds fixed).
def config_points(name):
    """Return (D, K list, description) for a named workload."""
    if name == "unif2d_50k":
        return uniform(50_000, 2, seed=1), [5], "uniform [0,100)^2, N=5e4"
    if name == "expo2d_2m":
        return exponential(2_000_000, 2, seed=2), [1, 8, 32, 64], "exponential(40) 2-D, N=2e6"
    if name == "expo4d_2m":
        return exponential(2_000_000, 4, seed=3), [1, 8, 32, 64], "exponential(40) 4-D, N=2e6"
    if name == "unif6d_5m":
        return uniform(5_000_000, 6, seed=4), [32], "uniform [0,100)^6, N=5e6"
    if name == "clustered2d_20m":
        return clustered(20_000_000, seed=5), [16], "clustered 2-D catalogue-shaped, N=2e7"
    raise KeyError(name)
