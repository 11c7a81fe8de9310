"""Path solvers of libccm against the oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import operators as ops
from gpu_util import need_gpu, dev, host, graph_dev, rel

pytestmark = pytest.mark.gpu

QS = [1.0, 2.0, np.inf]
METHODS = {"ssnal": 0, "admm": 1, "ama": 2}


def _opts(ccm, method, **kw):
    return ccm.ccm_default_options(method=METHODS[method], **kw)


def _certify(A, src, dst, w, g, q, X, U, tol):
    """Oracle KKT certificate of a GPU (X, U) pair."""
    B = oracle.incidence(src, dst, A.shape[0])
    res = ops.kkt_residuals(X, U, A, B, g * w, q)
    assert res["kkt"] <= tol * 1.0001, res
    return res


def _compare_path(A, src, dst, w, gammas, q, method, tol_gpu, tol_oracle=1e-10,
                  x_tol=1e-5, opts_kw=None):
    torch, ccm = need_gpu()
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), gammas, q, tol_gpu,
                             opts=_opts(ccm, method, **(opts_kw or {})), want_U=True)
    ref = oracle.solve_path(A, src, dst, w, gammas, q, tol_oracle, method="ssnal")
    S = oracle.fusion_scale(A)
    for t, g in enumerate(gammas):
        X = host(out["X"][t])
        U = host(out["U"][t])
        assert out["status"][t] == 0, (t, g, out["status"][t], out["kkt"][t])
        _certify(A, src, dst, w, g, q, X, U, tol_gpu)
        assert rel(X, ref["X"][t]) <= x_tol, (t, g, rel(X, ref["X"][t]))
        # labels: bit-exact when every edge has a clear fusion margin
        mg = oracle.fusion_margins(ref["X"][t], ref["U"][t], src, dst, w, g, q, S)
        if mg.min() > 1e-4:
            assert np.array_equal(host(out["labels"][t]), ref["labels"][t]), (t, g)
            assert out["n_clusters"][t] == ref["n_clusters"][t]
    return out, ref


@pytest.mark.parametrize("method", ["ssnal", "admm"])
def test_blobs2d_path(method):
    A, _ = synthdata.blobs2d()
    src, dst, w, *_ = oracle.knn_graph(A, 10, 0.5)
    gammas = synthdata.gamma_grid(-3, 1, 10)
    _compare_path(A, src, dst, w, gammas, 2.0, method, 1e-6, x_tol=1e-5)


@pytest.mark.parametrize("q", QS)
def test_small_path_all_q(q):
    A, _ = synthdata.mixture64(n_per=40, d=8, n_blobs=4)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    gammas = synthdata.gamma_grid(-2, 1, 6)
    _compare_path(A, src, dst, w, gammas, q, "ssnal", 1e-8, x_tol=1e-6)


@pytest.mark.parametrize("q", QS)
def test_ama_small(q):
    A, _ = synthdata.blobs2d(n_per=15)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    gammas = synthdata.gamma_grid(-2, 0.5, 4)
    _compare_path(A, src, dst, w, gammas, q, "ama", 1e-7, x_tol=1e-5)


@pytest.mark.parametrize("d", [3, 64, 130])
def test_ragged_dims(d):
    A, _ = synthdata.mixture64(n_per=30, d=d, n_blobs=5, seed=7 + d)
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    gammas = [0.0, 0.05, 0.5, 5.0]
    _compare_path(A, src, dst, w, gammas, 2.0, "ssnal", 1e-8, x_tol=1e-6)


def test_gamma_zero_and_no_edges():
    torch, ccm = need_gpu()
    A = np.random.default_rng(0).normal(size=(20, 3))
    out = ccm.ccm_solve_path(dev(A), dev(np.zeros(0, np.int32)), dev(np.zeros(0, np.int32)),
                             dev(np.zeros(0)), [0.0, 1.0], 2.0, 1e-6)
    for t in range(2):
        assert np.array_equal(host(out["X"][t]), A)
        assert out["n_clusters"][t] == 20
        assert np.array_equal(host(out["labels"][t]), np.arange(20))


def test_noncanonical_edges_are_merged():
    torch, ccm = need_gpu()
    A, _ = synthdata.blobs2d(n_per=10)
    src, dst, w, *_ = oracle.knn_graph(A, 4, 0.5)
    # reversed duplicates with split weights, plus a self loop and a zero weight
    s2 = np.concatenate([dst, src, [3], [1]]).astype(np.int32)
    d2 = np.concatenate([src, dst, [3], [2]]).astype(np.int32)
    w2 = np.concatenate([0.25 * w, 0.75 * w, [1.0], [0.0]])
    g = [0.1, 0.4]
    out = ccm.ccm_solve_path(dev(A), *graph_dev(s2, d2, w2), g, 2.0, 1e-9)
    ref = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-9)
    for t in range(2):
        assert rel(host(out["X"][t]), host(ref["X"][t])) <= 1e-7


def test_deterministic():
    torch, ccm = need_gpu()
    A, _ = synthdata.mixture64(n_per=100, d=16, n_blobs=5)
    src, dst, w, *_ = oracle.knn_graph(A, 8, None)
    g = synthdata.gamma_grid(-2, 1, 5)
    a = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-7)
    b = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-7)
    assert torch.equal(a["X"], b["X"])
    assert np.array_equal(a["kkt"], b["kkt"])


def test_invalid_arguments():
    torch, ccm = need_gpu()
    A = dev(np.zeros((5, 2)))
    s, d_, w = graph_dev([0, 1], [1, 2], [1.0, 1.0])
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [0.1], 3.0, 1e-6)
    assert e.value.status == 2
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [-0.1], 2.0, 1e-6)
    assert e.value.status == 1
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [0.1], 2.0, 0.0)
    assert e.value.status == 1
    bad_s, bad_d, bad_w = graph_dev([0, 7], [1, 2], [1.0, 1.0])
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, bad_s, bad_d, bad_w, [0.1], 2.0, 1e-6)
    assert e.value.status == 1
    s3, d3, w3 = graph_dev([0, 1], [1, 2], [1.0, -1.0])
    with pytest.raises(ccm.CcmError):
        ccm.ccm_solve_path(A, s3, d3, w3, [0.1], 2.0, 1e-6)
    An = np.zeros((5, 2))
    An[2, 1] = np.nan
    with pytest.raises(ccm.CcmError):
        ccm.ccm_solve_path(dev(An), s, d_, w, [0.1], 2.0, 1e-6)


def test_max_iter_status_and_time_budget():
    torch, ccm = need_gpu()
    A, _ = synthdata.blobs2d(n_per=20)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    o = ccm.ccm_default_options(max_outer=1, max_newton=1)
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [0.3], 2.0, 1e-12, opts=o)
    assert out["status"][0] == 1
    assert np.all(np.isfinite(host(out["X"][0])))
    o = ccm.ccm_default_options(time_budget_s=1e-9)
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [0.3, 0.6], 2.0, 1e-12, opts=o)
    assert out["status"][0] == 2
