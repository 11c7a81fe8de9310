"""Pins for the oracle solvers (SSNAL, ADMM, fast AMA): closed forms,
invariants, brute force and cross-checks.  CPU only."""
import numpy as np
import pytest
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree
import scipy.sparse as sp

import oracle
import synthdata
from oracle import operators as ops
from oracle.brute import dual_slsqp, primal_value, proj_l1_bisection

QS = [1.0, 2.0, np.inf]
SOLVERS = ["ssnal", "admm", "ama", "hpr"]


def solve(method, A, src, dst, w, g, q, tol=1e-10):
    if method == "ssnal":
        X, U, _, info = oracle.ssnal(A, src, dst, w, g, q, tol)
    elif method == "admm":
        X, U, _, info = oracle.admm(A, src, dst, w, g, q, tol)
    elif method == "hpr":
        X, U, _, info = oracle.hpr(A, src, dst, w, g, q, tol)
    else:
        X, U, info = oracle.ama(A, src, dst, w, g, q, tol)
    return X, U, info


def two_point_prox(delta, t, q):
    """prox of t||.||_q at delta, from textbook formulas (block / scalar soft
    threshold; for q = inf, delta minus the l1-ball projection found by
    bisection)."""
    if q == 2.0:
        nd = np.linalg.norm(delta)
        return delta * max(0.0, 1.0 - t / nd)
    if q == 1.0:
        return np.sign(delta) * np.maximum(np.abs(delta) - t, 0.0)
    return delta - proj_l1_bisection(delta, t)


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("q", QS)
def test_gamma_zero_gives_identity(method, q):
    A, _ = synthdata.blobs2d(n_per=5)
    src, dst, w = synthdata.random_graph(A.shape[0], 40, seed=3)
    X, U, info = solve(method, A, src, dst, w, 0.0, q)
    assert np.array_equal(X, A)
    assert np.all(U == 0)
    assert info["kkt"] == 0.0


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("g", [0.05, 0.3, 0.9, 5.0])
def test_two_point_closed_form(method, q, g):
    rng = np.random.default_rng(11)
    A = rng.normal(size=(2, 3)) * 2
    src, dst, w = np.array([0], np.int32), np.array([1], np.int32), np.array([0.7])
    X, U, info = solve(method, A, src, dst, w, g, q)
    delta = two_point_prox(A[0] - A[1], 2 * g * 0.7, q)
    assert np.allclose(X[0] - X[1], delta, atol=1e-8)
    assert np.allclose(X[0] + X[1], A[0] + A[1], atol=1e-12)
    # labels: fused iff 2 gamma w >= ||a1 - a2||_{q*} (the prox of t||.||_q
    # vanishes exactly on the dual-norm ball of radius t)
    lab, nc = oracle.cluster_labels(X, src, dst, 2, oracle.fusion_scale(A))
    fused = 2 * g * 0.7 >= ops.row_norms((A[0] - A[1])[None], ops.dual_exponent(q))[0]
    assert (nc == 1) == fused


@pytest.mark.parametrize("q", QS)
def test_two_point_labels_at_threshold(q):
    rng = np.random.default_rng(12)
    A = rng.normal(size=(2, 4))
    src, dst, w = np.array([0], np.int32), np.array([1], np.int32), np.array([1.0])
    gth = ops.row_norms((A[0] - A[1])[None], ops.dual_exponent(q))[0] / 2.0
    for fac, expect in ((0.98, 2), (1.02, 1)):
        X, U, _ = solve("ssnal", A, src, dst, w, fac * gth, q, tol=1e-11)
        _, nc = oracle.cluster_labels(X, src, dst, 2, oracle.fusion_scale(A))
        assert nc == expect


def _components(n, src, dst):
    G = sp.coo_matrix((np.ones(len(src)), (src, dst)), shape=(n, n))
    return connected_components(G, directed=False)[1]


@pytest.mark.parametrize("q", QS)
def test_centroid_preserved(q):
    """1^T B^T = 0 per component, so sum_{i in comp} x_i = sum a_i: at every
    ADMM iterate (its X-update is an exact solve with I + sigma B^T B), and
    for SSNAL's final point up to its dual residual (its Newton directions
    come from preconditioned CG, which only preserves sums in the limit)."""
    A, _ = synthdata.blobs2d(n_per=8)
    n = A.shape[0]
    src, dst, w, *_ = oracle.knn_graph(A, 3, 0.5)
    comp = _components(n, src, dst)
    target = np.array([A[comp == c].sum(0) for c in range(comp.max() + 1)])
    seen = []

    def dev(X):
        got = np.array([X[comp == c].sum(0) for c in range(comp.max() + 1)])
        return np.abs(got - target).max() / (1 + np.abs(target).max())

    oracle.admm(A, src, dst, w, 0.2, q, 1e-8, callback=lambda X: seen.append(dev(X)))
    assert len(seen) > 0
    assert max(seen) <= 1e-12
    # HPR solves the same X system exactly at every iterate
    seen.clear()
    oracle.hpr(A, src, dst, w, 0.2, q, 1e-8, callback=lambda X: seen.append(dev(X)))
    assert len(seen) > 0
    assert max(seen) <= 1e-12
    X, U, _, info = oracle.ssnal(A, src, dst, w, 0.2, q, 1e-10)
    B = oracle.incidence(src, dst, n)
    resid = X - A + B.T @ U
    for c in range(comp.max() + 1):
        bound = np.sqrt((comp == c).sum()) * np.linalg.norm(resid[comp == c]) + 1e-12
        assert np.abs(X[comp == c].sum(0) - target[c]).max() <= bound


def full_fusion_certificate(A, src, dst, w, q):
    """Spanning-tree flows U with A - B^T U = component means, and the
    smallest gamma for which they are feasible (SURVEY pin P4)."""
    n, d = A.shape
    m = len(src)
    comp = _components(n, src, dst)
    # maximum weight spanning forest
    W = sp.coo_matrix((-np.asarray(w), (src, dst)), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(W).tocoo()
    key = {(min(a, b), max(a, b)): l for l, (a, b) in enumerate(zip(src, dst))}
    tree = [key[(min(a, b), max(a, b))] for a, b in zip(T.row, T.col)]
    means = np.array([A[comp == c].mean(0) for c in range(comp.max() + 1)])
    C = A - means[comp]
    U = np.zeros((m, d))
    adj = {i: [] for i in range(n)}
    for l in tree:
        adj[int(src[l])].append((int(dst[l]), l))
        adj[int(dst[l])].append((int(src[l]), l))
    for l in tree:
        i, j = int(src[l]), int(dst[l])
        # side of i after removing l
        seen = {i}
        stack = [i]
        while stack:
            v = stack.pop()
            for u, ll in adj[v]:
                if ll != l and u not in seen:
                    seen.add(u)
                    stack.append(u)
        U[l] = C[list(seen)].sum(0)
    gtree = max(ops.row_norms(U[tree], ops.dual_exponent(q)) / np.asarray(w)[tree])
    return U, gtree, means[comp]


@pytest.mark.parametrize("q", QS)
def test_full_fusion_certificate_and_solvers(q):
    A, _ = synthdata.blobs2d(n_per=6)
    src, dst, w, *_ = oracle.knn_graph(A, 4, 0.5)
    U, gtree, M = full_fusion_certificate(A, src, dst, w, q)
    B = oracle.incidence(src, dst, A.shape[0])
    # the certificate itself: flows reproduce the component means exactly
    assert np.allclose(A - B.T @ U, M, atol=1e-12)
    g = 1.2 * gtree
    res = ops.kkt_residuals(M, U, A, B, g * w, q)
    assert res["kkt"] <= 1e-13 and res["eta"] <= 1e-13
    for method in SOLVERS:
        X, _, info = solve(method, A, src, dst, w, g, q, tol=1e-9)
        assert np.abs(X - M).max() <= 1e-6 * (1 + np.abs(M).max()), method


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_brute_force(q, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 7))
    d = int(rng.integers(1, 4))
    A = rng.normal(size=(n, d))
    src, dst, w = synthdata.random_graph(n, 2 * n, seed=seed)
    g = float(rng.uniform(0.05, 0.6))
    Xb, Ub = dual_slsqp(A, src, dst, w, g, q)
    X, U, _, info = oracle.ssnal(A, src, dst, w, g, q, 1e-11)
    assert np.allclose(X, Xb, atol=2e-6)
    fx = primal_value(X, A, src, dst, w, g, q)
    assert fx <= primal_value(Xb, A, src, dst, w, g, q) + 1e-9
    # no random perturbation improves the SSNAL point
    for _ in range(50):
        assert primal_value(X + 1e-4 * rng.normal(size=X.shape), A, src, dst, w, g, q) >= fx - 1e-12


@pytest.mark.parametrize("q", QS)
def test_d1_complete_graph_closed_form(q):
    # d = 1, complete graph, unit weights: before any merge
    # x_(k) = a_(k) - gamma (2k - n - 1) in sorted order (Hocking et al. 2011)
    a = np.array([0.0, 1.0, 2.5, 3.1, 5.0, 6.2])
    rng = np.random.default_rng(3)
    perm = rng.permutation(a.size)
    A = a[perm][:, None]
    n = a.size
    src, dst = np.triu_indices(n, 1)
    w = np.ones(src.size)
    g = 0.1  # smallest gap 0.6 > 2 gamma
    X, _, _, _ = oracle.ssnal(A, src.astype(np.int32), dst.astype(np.int32), w, g, q, 1e-12)
    order = np.argsort(A[:, 0])
    k = np.arange(1, n + 1)
    expect = np.sort(a) - g * (2 * k - n - 1)
    assert np.allclose(X[order, 0], expect, atol=1e-9)


def test_d1_all_q_coincide():
    A, _ = synthdata.blobs2d(n_per=6)
    A = A[:, :1].copy()
    src, dst, w, *_ = oracle.knn_graph(A, 4, 0.5)
    Xs = [oracle.ssnal(A, src, dst, w, 0.15, q, 1e-11)[0] for q in QS]
    assert np.allclose(Xs[0], Xs[1], atol=1e-8) and np.allclose(Xs[1], Xs[2], atol=1e-8)


def test_q1_separable_over_columns():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(15, 3))
    src, dst, w = synthdata.random_graph(15, 40, seed=5)
    X, *_ = oracle.ssnal(A, src, dst, w, 0.2, 1.0, 1e-11)
    for c in range(3):
        Xc, *_ = oracle.ssnal(A[:, c:c + 1].copy(), src, dst, w, 0.2, 1.0, 1e-11)
        assert np.allclose(X[:, c], Xc[:, 0], atol=1e-8)


@pytest.mark.parametrize("q", QS)
def test_equivariances(q):
    rng = np.random.default_rng(6)
    n, d = 14, 3
    A = rng.normal(size=(n, d))
    src, dst, w = synthdata.random_graph(n, 35, seed=6)
    g = 0.25
    X, *_ = oracle.ssnal(A, src, dst, w, g, q, 1e-11)
    # translation
    c = rng.normal(size=d)
    Xt, *_ = oracle.ssnal(A + c, src, dst, w, g, q, 1e-11)
    assert np.allclose(Xt, X + c, atol=1e-8)
    # scaling X*(sA, s gamma) = s X*(A, gamma)
    Xs, *_ = oracle.ssnal(2.5 * A, src, dst, w, 2.5 * g, q, 1e-11)
    assert np.allclose(Xs, 2.5 * X, atol=1e-7)
    # permutation of points
    perm = rng.permutation(n)
    inv = np.argsort(perm)
    s2, d2, w2 = oracle.canonicalize_edges(inv[src], inv[dst], w)
    Xp, *_ = oracle.ssnal(A[perm], s2, d2, w2, g, q, 1e-11)
    assert np.allclose(Xp, X[perm], atol=1e-8)
    if q == 2.0:
        Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
        Xr, *_ = oracle.ssnal(A @ Q, src, dst, w, g, q, 1e-11)
        assert np.allclose(Xr, X @ Q, atol=1e-8)


@pytest.mark.parametrize("q", QS)
def test_solvers_agree_on_path(q):
    A, _ = synthdata.blobs2d(n_per=15)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    gs = synthdata.gamma_grid(-2, 0.5, 5)
    ref = oracle.solve_path(A, src, dst, w, gs, q, 1e-9, method="ssnal")
    for method in ("admm", "ama", "hpr"):
        out = oracle.solve_path(A, src, dst, w, gs, q, 1e-9, method=method)
        for t in range(len(gs)):
            rel = np.linalg.norm(out["X"][t] - ref["X"][t]) / np.linalg.norm(ref["X"][t])
            assert rel <= 1e-6, (method, t, rel)
            assert np.array_equal(out["labels"][t], ref["labels"][t])


@pytest.mark.parametrize("q", QS)
def test_value_function_monotone_concave_envelope(q):
    A, _ = synthdata.blobs2d(n_per=10)
    src, dst, w, *_ = oracle.knn_graph(A, 5, 0.5)
    B = oracle.incidence(src, dst, A.shape[0])
    gs = np.linspace(0.02, 0.4, 8)
    f = []
    slope = []
    for g in gs:
        X, U, _, info = oracle.ssnal(A, src, dst, w, g, q, 1e-11)
        f.append(ops.primal_objective(X, A, B, g * w, q))
        slope.append(float((w * ops.row_norms(B @ X, q)).sum()))
    f = np.array(f)
    assert np.all(np.diff(f) >= -1e-10)
    # concavity: secant slopes decrease; envelope slope lies between
    sec = np.diff(f) / np.diff(gs)
    assert np.all(np.diff(sec) <= 1e-8)
    for t in range(len(gs) - 1):
        assert slope[t] >= sec[t] - 1e-6 and slope[t + 1] <= sec[t] + 1e-6


def test_path_continuity():
    A, _ = synthdata.blobs2d(n_per=10)
    src, dst, w, *_ = oracle.knn_graph(A, 5, 0.5)
    g = 0.3
    X0, *_ = oracle.ssnal(A, src, dst, w, g, 2.0, 1e-11)
    d = []
    for h in (1e-2, 1e-3, 1e-4):
        Xh, *_ = oracle.ssnal(A, src, dst, w, g + h, 2.0, 1e-11)
        d.append(np.linalg.norm(Xh - X0))
    assert d[0] > d[1] > d[2]
    assert d[2] < 1e-2 * d[0] * 10
