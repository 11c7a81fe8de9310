"""Seeded synthetic inputs for the convex clustering workloads.

This module only draws random numbers and arranges them into point sets,
gamma grids, targets and random test graphs.  It holds none of the
clustering method's arithmetic (no k-NN search, no weights, no solver):
both the CPU oracle and the GPU library consume what it produces, and it
imports neither of them.

Every generator is deterministic in its seed.  The draw order inside each
recipe is fixed (centres, then assignments, then noise, then a shuffle) so
that two processes that ask for the same workload get bit-identical arrays.

Workload recipes (sizes as used by the tests and the benchmark):

* ``blobs2d``      -- 4 isotropic Gaussian blobs of 50 points in 2-D,
                      sigma 0.5, centres uniform in [-5, 5]^2.
* ``mixture64``    -- 10 Gaussians of 1000 points in 64-D, sigma 1,
                      centres N(0, 25 I).
* ``images784``    -- 10 classes of image-shaped data in 784-D: class
                      prototypes uniform in [0, 1], pixel = prototype +
                      N(0, 0.1^2), clipped to [0, 1] and quantised to k/255
                      with k = rint(255 p) (round half to even).
* ``instances``    -- many independent blob instances of uneven n, d, q.
* ``mixture32``    -- 8 Gaussians of 2500 points in 32-D with N(0, I)
                      regression targets (the differentiated workload).

The paper evaluates on public datasets (LIBRAS, COIL-20, LUNG, MNIST);
these synthetic sets stand in for them and reproduce none of their records.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian_blobs",
    "blobs2d",
    "mixture64",
    "images784",
    "mixture32",
    "instances",
    "gamma_grid",
    "random_graph",
    "chain_graph",
    "WORKLOADS",
]


def _shuffle(rng, *arrays):
    perm = rng.permutation(arrays[0].shape[0])
    return tuple(a[perm] for a in arrays)


def gaussian_blobs(rng, n_blobs, n_per, d, sigma, centre_kind, centre_scale):
    """Balanced isotropic Gaussian blobs, shuffled.

    centre_kind 'uniform': centres ~ U[-centre_scale, centre_scale]^d;
    centre_kind 'normal' : centres ~ N(0, centre_scale^2 I).
    Returns (A float64 [n, d], y int32 [n]).
    """
    if centre_kind == "uniform":
        centres = rng.uniform(-centre_scale, centre_scale, size=(n_blobs, d))
    elif centre_kind == "normal":
        centres = rng.normal(0.0, centre_scale, size=(n_blobs, d))
    else:
        raise ValueError(centre_kind)
    y = np.repeat(np.arange(n_blobs, dtype=np.int32), n_per)
    noise = rng.normal(0.0, sigma, size=(n_blobs * n_per, d))
    A = centres[y] + noise
    A, y = _shuffle(rng, A, y)
    return np.ascontiguousarray(A, dtype=np.float64), np.ascontiguousarray(y)


def blobs2d(seed=1001, n_per=50):
    """4 blobs x n_per points in 2-D, sigma 0.5, centres U[-5,5]^2."""
    rng = np.random.default_rng(seed)
    return gaussian_blobs(rng, 4, n_per, 2, 0.5, "uniform", 5.0)


def mixture64(seed=1002, n_per=1000, d=64, n_blobs=10):
    """n_blobs Gaussians x n_per points in d dims, sigma 1, centres N(0, 25 I)."""
    rng = np.random.default_rng(seed)
    return gaussian_blobs(rng, n_blobs, n_per, d, 1.0, "normal", 5.0)


def mixture32(seed=1005, n_per=2500, d=32, n_blobs=8):
    """8 Gaussians x 2500 points in 32-D (sigma 1, centres N(0, 25 I)) plus
    targets t_i ~ N(0, I).  Returns (A, y, T)."""
    rng = np.random.default_rng(seed)
    A, y = gaussian_blobs(rng, n_blobs, n_per, d, 1.0, "normal", 5.0)
    T = rng.normal(0.0, 1.0, size=A.shape)
    return A, y, np.ascontiguousarray(T)


def images784(seed=1003, n_per=10000, d=784, n_classes=10, noise=0.1):
    """Image-shaped classes quantised to k/255.  Returns (A, y, K) where K
    holds the integer codes k in [0, 255] (uint8) and A = K / 255."""
    rng = np.random.default_rng(seed)
    protos = rng.uniform(0.0, 1.0, size=(n_classes, d))
    y = np.repeat(np.arange(n_classes, dtype=np.int32), n_per)
    n = n_classes * n_per
    # draw noise in row blocks so peak memory stays modest at n = 1e5
    K = np.empty((n, d), dtype=np.uint8)
    blk = 8192
    for s in range(0, n, blk):
        e = min(n, s + blk)
        p = protos[y[s:e]] + rng.normal(0.0, noise, size=(e - s, d))
        K[s:e] = np.rint(255.0 * np.clip(p, 0.0, 1.0)).astype(np.uint8)
    K, y = _shuffle(rng, K, y)
    A = K.astype(np.float64) / 255.0
    return np.ascontiguousarray(A), np.ascontiguousarray(y), np.ascontiguousarray(K)


def instances(seed=1004, count=512, n_lo=100, n_hi=5000, dims=(2, 8, 32, 128),
              blobs_lo=2, blobs_hi=12, qs=(1.0, 2.0, np.inf)):
    """Independent blob instances of uneven size.  Each entry is a dict with
    keys A, n, d, q, n_blobs.  n ~ U{n_lo..n_hi}, d ~ U(dims), blobs ~
    U{blobs_lo..blobs_hi}, q ~ U(qs); centres U[-5,5]^d, sigma 0.5.  Point
    counts are split as evenly as possible over the blobs."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(dims[int(rng.integers(0, len(dims)))])
        nb = int(rng.integers(blobs_lo, blobs_hi + 1))
        q = float(qs[int(rng.integers(0, len(qs)))])
        centres = rng.uniform(-5.0, 5.0, size=(nb, d))
        y = (np.arange(n) % nb).astype(np.int32)
        A = centres[y] + rng.normal(0.0, 0.5, size=(n, d))
        A, y = _shuffle(rng, A, y)
        out.append(dict(A=np.ascontiguousarray(A), y=y, n=n, d=d, q=q, n_blobs=nb))
    return out


def gamma_grid(lo_exp, hi_exp, count):
    """count values log-spaced from 10^lo_exp to 10^hi_exp (ascending)."""
    return np.logspace(lo_exp, hi_exp, count)


def random_graph(n, m, seed, w_lo=0.1, w_hi=1.0):
    """m distinct undirected edges (i < j) drawn uniformly among the n(n-1)/2
    pairs, with weights ~ U[w_lo, w_hi].  Returned sorted by (i, j)."""
    rng = np.random.default_rng(seed)
    total = n * (n - 1) // 2
    m = min(m, total)
    keys = set()
    while len(keys) < m:
        i = rng.integers(0, n, size=2 * (m - len(keys)) + 8)
        j = rng.integers(0, n, size=i.shape[0])
        for a, b in zip(i.tolist(), j.tolist()):
            if a != b:
                keys.add((min(a, b), max(a, b)))
            if len(keys) >= m:
                break
    e = np.array(sorted(keys), dtype=np.int32).reshape(-1, 2)
    w = rng.uniform(w_lo, w_hi, size=e.shape[0])
    return e[:, 0].copy(), e[:, 1].copy(), w


def chain_graph(n, seed=None, w=None):
    """Path graph 0-1-2-...-(n-1); unit weights unless w is given or a seed
    asks for U[0.5, 1.5] weights."""
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    if w is None:
        if seed is None:
            w = np.ones(n - 1)
        else:
            w = np.random.default_rng(seed).uniform(0.5, 1.5, size=n - 1)
    return src, dst, np.asarray(w, dtype=np.float64)


# name -> (generator, k, phi, gammas, q list, description)
WORKLOADS = {
    "blobs2d_n200": dict(points=blobs2d, k=10, phi=0.5, gammas=(-3, 1, 10), q=(2.0,),
                         desc="n=200 d=2 4 blobs, k=10, w=exp(-0.5 d^2), q=2, 10 gammas in [1e-3,1e1]"),
    "mixture64_n10000": dict(points=mixture64, k=10, phi=None, gammas=(-3, 2, 20), q=(2.0,),
                             desc="n=10000 d=64 10 Gaussians, k=10, phi=1/median kNN d^2, q=2, 20 gammas in [1e-3,1e2]"),
    "images784_n100000": dict(points=images784, k=10, phi=None, gammas=(-3, 1, 15), q=(1.0, 2.0, np.inf),
                              desc="n=100000 d=784 10 image classes quantised to k/255, k=10, q in {1,2,inf}, 15 gammas"),
    "mixture32_n20000": dict(points=mixture32, k=10, phi=None, gammas=None, q=(2.0,),
                             desc="n=20000 d=32 8 Gaussians, k=10, q=2, gamma=0.5, loss sum ||x_i - t_i||^2"),
}
