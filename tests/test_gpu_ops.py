"""Edge operators of libccm against the oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import operators as ops
from gpu_util import need_gpu, dev, host, graph_dev, rel

pytestmark = pytest.mark.gpu

QS = [1.0, 2.0, np.inf]
DIMS = [1, 2, 3, 5, 8, 31, 64, 65, 130, 784]


def _graph(n, m, seed):
    """Random graph plus a hub (vertex 1 joined to every 2nd vertex, degree far
    above any vertex-window width) and isolated vertices (the last three)."""
    src, dst, w = synthdata.random_graph(n - 3, m, seed)
    rng = np.random.default_rng(seed + 1)
    hub = [(1, j) for j in range(2, n - 3, 2)]
    keys = {(int(a), int(b)): float(c) for a, b, c in zip(src, dst, w)}
    for a, b in hub:
        keys.setdefault((a, b), float(rng.uniform(0.1, 1.0)))
    e = sorted(keys)
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    w = np.array([keys[k] for k in e])
    return src, dst, w


@pytest.mark.parametrize("d", DIMS)
def test_gather_exact(d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(d)
    n, m = 300, 1700
    X = rng.normal(size=(n, d))
    src, dst, w = _graph(n, m, d)
    B = oracle.incidence(src, dst, n)
    Y = host(ccm.ccm_op_gather(dev(X), *graph_dev(src, dst, w)[:2]))
    assert np.array_equal(Y, B @ X)  # one subtraction per entry: bit-exact


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("d", DIMS)
def test_project_and_prox(q, d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(100 + d)
    m = 2049  # several blocks and a ragged tail
    Y = rng.normal(size=(m, d)) * rng.uniform(0.1, 3.0, size=(m, 1))
    w = rng.uniform(0.2, 1.5, size=m)
    g = 0.7
    P = host(ccm.ccm_op_project(dev(Y), dev(w), g, q))
    Pr = ops.project(Y, g * w, q)
    assert np.allclose(P, Pr, rtol=1e-13, atol=1e-13)
    Z = host(ccm.ccm_op_prox(dev(Y), dev(w), g, q))
    assert np.allclose(Z, Y - Pr, rtol=1e-13, atol=1e-13)
    # feasibility of the GPU projection in the dual norm
    nd = ops.row_norms(P, ops.dual_exponent(q))
    assert np.all(nd <= g * w * (1 + 1e-12))


@pytest.mark.parametrize("d", [1, 3, 64, 130])
def test_scatter_matches_transpose(d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(200 + d)
    n, m = 513, 3000
    src, dst, w = _graph(n, m, 7 + d)
    Z = rng.normal(size=(len(src), d))
    B = oracle.incidence(src, dst, n)
    out = host(ccm.ccm_op_scatter(dev(Z), dev(src.astype(np.int32)), dev(dst.astype(np.int32)), n))
    ref = B.T @ Z
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-12)
    # adjointness with the gather on the device
    X = rng.normal(size=(n, d))
    Y = host(ccm.ccm_op_gather(dev(X), dev(src.astype(np.int32)), dev(dst.astype(np.int32))))
    lhs, rhs = float((Y * Z).sum()), float((X * out).sum())
    assert abs(lhs - rhs) <= 1e-11 * (1 + abs(lhs))


def test_scatter_isolated_vertices_and_empty_graph():
    torch, ccm = need_gpu()
    n, d = 50, 4
    src = np.array([3, 7], np.int32)
    dst = np.array([9, 40], np.int32)
    Z = np.arange(8, dtype=np.float64).reshape(2, 4)
    out = host(ccm.ccm_op_scatter(dev(Z), dev(src), dev(dst), n))
    ref = oracle.incidence(src, dst, n).T @ Z
    assert np.array_equal(out, ref)
    out0 = host(ccm.ccm_op_scatter(dev(np.zeros((0, d))), dev(np.zeros(0, np.int32)),
                                   dev(np.zeros(0, np.int32)), n))
    assert np.all(out0 == 0)


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("d", [1, 2, 7, 64, 100, 784])
def test_hess_matvec(q, d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(300 + d)
    n, m = 400, 2200
    src, dst, w = _graph(n, m, 11 + d)
    X = rng.normal(size=(n, d))
    U = rng.normal(size=(len(src), d)) * 0.3
    V = rng.normal(size=(n, d))
    g, sig = 0.8, 2.5
    out, ms = ccm.ccm_op_hess_matvec(dev(X), dev(U), *graph_dev(src, dst, w), g, sig, q, dev(V))
    B = oracle.incidence(src, dst, n)
    Y = U + sig * (B @ X)
    ref = V + sig * (B.T @ ops.jacobian_apply(Y, g * w, q, B @ V))
    assert rel(host(out), ref) <= 1e-12


@pytest.mark.parametrize("q", QS)
def test_kkt_evaluator(q):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(400)
    n, d = 300, 6
    A = rng.normal(size=(n, d))
    src, dst, w = _graph(n, 1500, 13)
    X = A + 0.1 * rng.normal(size=(n, d))
    U = rng.normal(size=(len(src), d)) * 0.2
    g = 0.3
    got = ccm.ccm_kkt(dev(A), dev(X), dev(U), *graph_dev(src, dst, w), g, q)
    B = oracle.incidence(src, dst, n)
    ref = ops.kkt_residuals(X, U, A, B, g * w, q)
    for k in ("R_D", "R_C", "R_U", "eta", "f_p", "f_d"):
        assert abs(got[k] - ref[k]) <= 1e-11 * (1 + abs(ref[k])), k


def test_labels_match_oracle():
    torch, ccm = need_gpu()
    rng = np.random.default_rng(500)
    n, d = 1000, 3
    A = rng.normal(size=(n, d))
    src, dst, w = _graph(n, 4000, 17)
    # X: points of a few random groups collapsed to group means
    grp = rng.integers(0, 60, size=n)
    X = A.copy()
    for c in range(60):
        X[grp == c] = A[grp == c].mean(0)
    lab, nc = ccm.ccm_labels(dev(A), dev(X), *graph_dev(src, dst, w)[:2])
    ref, nref = oracle.cluster_labels(X, src, dst, n, oracle.fusion_scale(A))
    assert nc == nref
    assert np.array_equal(host(lab), ref)


@pytest.mark.parametrize("d", [2, 64, 70])
def test_knn_graph_matches_oracle(d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(600 + d)
    n = 777
    A = rng.normal(size=(n, d))
    A[5] = A[9]  # duplicate point: distance 0, weight 1
    for phi in (0.0, 0.5):
        src, dst, w, phi_used = ccm.ccm_build_knn_graph(dev(A), 10, phi)
        s_o, d_o, w_o, phi_o, _, _ = oracle.knn_graph(A, 10, phi if phi > 0 else None)
        assert phi_used == phi_o
        assert np.array_equal(host(src), s_o) and np.array_equal(host(dst), d_o)
        assert np.allclose(host(w), w_o, rtol=1e-14, atol=0)


def test_knn_quantised_images():
    torch, ccm = need_gpu()
    A, y, K = synthdata.images784(n_per=150, d=784, n_classes=4)
    src, dst, w, phi = ccm.ccm_build_knn_graph(dev(A), 10, 0.0)
    s_o, d_o, w_o, phi_o, _, _ = oracle.knn_graph(A, 10, None)
    assert phi == phi_o
    assert np.array_equal(host(src), s_o) and np.array_equal(host(dst), d_o)
    assert np.allclose(host(w), w_o, rtol=1e-14, atol=0)


def test_stream_copy():
    torch, ccm = need_gpu()
    a = torch.arange(1 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    ms = ccm.ccm_stream_copy(a, b, a.numel() * 8, repeats=3)
    assert torch.equal(a, b) and ms > 0


@pytest.mark.parametrize("d", [2, 5, 64])
def test_l1_ball_projection_tiny_radius(d):
    # radii below the rounding resolution of max |y_k|: the projection is 0
    # (regression: support pruning must not cycle to an infeasible point)
    torch, ccm = need_gpu()
    rng = np.random.default_rng(700 + d)
    m = 300
    Y = rng.normal(size=(m, d)) * 3.0
    w = 10.0 ** rng.uniform(-24, -12, size=m)
    w[::7] = rng.uniform(0.1, 1.0, size=w[::7].shape)  # and some ordinary radii
    g = 1e-3
    P = host(ccm.ccm_op_project(dev(Y), dev(w), g, np.inf))
    Pr = ops.project(Y, g * w, np.inf)
    assert np.allclose(P, Pr, rtol=1e-12, atol=1e-14)
    # the kept magnitudes are rounded differences |y_k| - theta, so the l1
    # norm can exceed a radius below the spacing of |y| by a few ulps of |y|
    slack = 4 * d * np.finfo(float).eps * np.abs(Y).max(1)
    assert np.all(np.abs(P).sum(1) <= g * w * (1 + 1e-12) + slack)


@pytest.mark.parametrize("case", ["images", "ties", "ragged"])
def test_knn_u8_exact_integer_distances(case):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(800)
    if case == "images":
        A, y, K = synthdata.images784(n_per=150, d=784, n_classes=4)
    elif case == "ties":
        K = rng.integers(0, 3, size=(500, 20)).astype(np.uint8)  # massive exact ties
    else:
        K = rng.integers(0, 256, size=(333, 70)).astype(np.uint8)
    scale = 1.0 / 255.0
    for phi in (0.0, 0.3):
        src, dst, w, phi_used = ccm.ccm_build_knn_graph_u8(dev(K), scale, 10, phi)
        s_o, d_o, w_o, phi_o, _, _ = oracle.knn_graph_u8(K, scale, 10, phi if phi > 0 else None)
        assert phi_used == phi_o
        assert np.array_equal(host(src), s_o) and np.array_equal(host(dst), d_o)
        assert np.allclose(host(w), w_o, rtol=1e-14, atol=0)


def test_knn_u8_rejects_bad_arguments():
    torch, ccm = need_gpu()
    K = torch.zeros((10, 2049), dtype=torch.uint8, device="cuda")
    with pytest.raises(ccm.CcmError):
        ccm.ccm_build_knn_graph_u8(K, 1.0, 3)
    with pytest.raises(ccm.CcmError):
        ccm.ccm_build_knn_graph_u8(K[:, :5].contiguous(), 0.0, 3)


def _big_hub_graph(n, seed, hub_deg):
    """Random sparse graph plus vertex 5 joined to hub_deg others.  For rows of
    d >= 33 values a window holds at most 256 incidences, so the hub's list
    is split over every row group of its workgroup and over several rounds
    of loads; for d = 3 it sits inside one large window."""
    rng = np.random.default_rng(seed)
    src, dst, w = synthdata.random_graph(n, 3 * n, seed)
    keys = {(int(a), int(b)): float(c) for a, b, c in zip(src, dst, w)}
    for j in rng.choice(np.arange(6, n), hub_deg, replace=False):
        keys.setdefault((5, int(j)), float(rng.uniform(0.1, 1.0)))
    e = sorted(keys)
    return (np.array([a for a, _ in e], np.int32), np.array([b for _, b in e], np.int32),
            np.array([keys[k] for k in e]))


@pytest.mark.parametrize("d", [3, 64, 130, 784])
def test_scatter_and_matvec_with_a_hub_longer_than_a_window(d):
    torch, ccm = need_gpu()
    rng = np.random.default_rng(1100 + d)
    n = 900
    src, dst, w = _big_hub_graph(n, 40 + d, 600)
    assert np.bincount(np.r_[src, dst], minlength=n).max() >= 600
    B = oracle.incidence(src, dst, n)
    Z = rng.normal(size=(len(src), d))
    out = host(ccm.ccm_op_scatter(dev(Z), dev(src), dev(dst), n))
    assert np.allclose(out, B.T @ Z, rtol=1e-13, atol=1e-12)
    for q in QS:
        X = rng.normal(size=(n, d))
        U = rng.normal(size=(len(src), d)) * 0.3
        V = rng.normal(size=(n, d))
        g, sig = 0.8, 2.5
        res, _ = ccm.ccm_op_hess_matvec(dev(X), dev(U), *graph_dev(src, dst, w), g, sig, q, dev(V))
        Y = U + sig * (B @ X)
        ref = V + sig * (B.T @ ops.jacobian_apply(Y, g * w, q, B @ V))
        assert rel(host(res), ref) <= 1e-12, q
