"""Paths solved with the locality order of the vertex kernels (GPU).

The library visits the points component by component, each in breadth-first
levels, when asked to (ccm_options.locality = 1) or for large problems; the
order changes only which rows are summed when, so every path must still
match the oracle.  These graphs are small, so the order is forced on."""
import numpy as np
import pytest

import oracle
import synthdata
from gpu_util import need_gpu, dev, host, graph_dev, rel
from test_gpu_solver import QS, _compare_path

pytestmark = pytest.mark.gpu


def _with_isolated(A, src, dst, w, extra, seed):
    """Appends `extra` points far from everything and with no edges."""
    rng = np.random.default_rng(seed)
    far = 1e3 + rng.normal(size=(extra, A.shape[1]))
    return np.vstack([A, far]), src, dst, w


@pytest.mark.parametrize("q", QS)
def test_locality_path_all_q(q):
    A, _ = synthdata.mixture64(n_per=40, d=8, n_blobs=4, seed=2201)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    A, src, dst, w = _with_isolated(A, src, dst, w, 3, 2202)
    gammas = synthdata.gamma_grid(-2, 1, 5)
    _compare_path(A, src, dst, w, gammas, q, "ssnal", 1e-8, x_tol=1e-6,
                  opts_kw=dict(locality=1))


@pytest.mark.parametrize("method", ["admm", "ama"])
def test_locality_first_order_methods(method):
    A, _ = synthdata.blobs2d(n_per=20, seed=2203)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    gammas = synthdata.gamma_grid(-2, 0.5, 4)
    _compare_path(A, src, dst, w, gammas, 2.0, method, 1e-7, x_tol=1e-5,
                  opts_kw=dict(locality=1))


@pytest.mark.parametrize("q", [2.0, np.inf])
def test_locality_hub_longer_than_a_window(q):
    rng = np.random.default_rng(2204)
    n, d = 600, 40
    A = rng.normal(size=(n, d))
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    keys = {(int(a), int(b)): float(c) for a, b, c in zip(src, dst, w)}
    # the hub is a late vertex, so its window is not first in vertex order
    hub = n - 7
    for j in rng.choice(np.arange(0, n - 10), 350, replace=False):
        keys.setdefault((int(j), hub), float(rng.uniform(0.05, 0.3)))
    e = sorted(keys)
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    w = np.array([keys[k] for k in e])
    assert np.bincount(np.r_[src, dst], minlength=n).max() >= 350
    _compare_path(A, src, dst, w, [0.01, 0.05], q, "ssnal", 1e-7, x_tol=1e-5,
                  opts_kw=dict(locality=1))


def test_locality_order_is_deterministic_and_agrees_with_input_order():
    torch, ccm = need_gpu()
    A, _ = synthdata.mixture64(n_per=120, d=16, n_blobs=5, seed=2205)
    src, dst, w, *_ = oracle.knn_graph(A, 8, None)
    g = synthdata.gamma_grid(-2, 1, 5)
    runs = [ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-9,
                               opts=ccm.ccm_default_options(locality=loc))
            for loc in (1, 1, 0)]
    a, b, c = runs
    assert torch.equal(a["X"], b["X"])
    assert np.array_equal(a["kkt"], b["kkt"])
    for t in range(len(g)):
        assert rel(host(a["X"][t]), host(c["X"][t])) <= 1e-7
        assert np.array_equal(host(a["labels"][t]), host(c["labels"][t]))
