"""Pins for the oracle's edge operators (operator identities, projections,
generalized Jacobians).  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import operators as ops
from oracle.brute import dense_incidence, proj_l1_bisection

QS = [1.0, 2.0, np.inf]


def _rand(m, d, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(m, d)) * scale
    r = rng.uniform(0.1, 2.0, size=m)
    return Y, r


def test_incidence_matches_python_loop():
    rng = np.random.default_rng(0)
    n, m = 9, 14
    src = rng.integers(0, n, m)
    dst = (src + 1 + rng.integers(0, n - 1, m)) % n
    B = oracle.incidence(src, dst, n).toarray()
    assert np.array_equal(B, dense_incidence(src, dst, n))


def test_adjointness_and_laplacian():
    rng = np.random.default_rng(1)
    n, m, d = 12, 30, 3
    src = rng.integers(0, n, m)
    dst = (src + 1 + rng.integers(0, n - 1, m)) % n
    B = oracle.incidence(src, dst, n)
    X = rng.normal(size=(n, d))
    Z = rng.normal(size=(m, d))
    lhs = float(((B @ X) * Z).sum())
    rhs = float((X * (B.T @ Z)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))
    # B^T B equals the (unweighted, multigraph) Laplacian degree - adjacency
    Lap = np.zeros((n, n))
    for a, b in zip(src, dst):
        Lap[a, a] += 1
        Lap[b, b] += 1
        Lap[a, b] -= 1
        Lap[b, a] -= 1
    assert np.allclose((B.T @ B).toarray(), Lap, atol=0)


@pytest.mark.parametrize("q", QS)
def test_projection_feasible_idempotent(q):
    Y, r = _rand(200, 7, 2, scale=2.0)
    P = ops.project(Y, r, q)
    nd = ops.row_norms(P, ops.dual_exponent(q))
    assert np.all(nd <= r * (1 + 1e-12))
    assert np.allclose(ops.project(P, r, q), P, atol=1e-14, rtol=0)


def test_l2_prox_is_block_soft_threshold():
    Y, r = _rand(100, 5, 3, scale=2.0)
    nrm = np.sqrt((Y * Y).sum(1))
    expect = Y * np.maximum(0.0, 1.0 - r / nrm)[:, None]
    assert np.allclose(ops.prox(Y, r, 2.0), expect, atol=1e-14)


def test_l1_prox_is_soft_threshold():
    Y, r = _rand(100, 5, 4, scale=2.0)
    expect = np.sign(Y) * np.maximum(np.abs(Y) - r[:, None], 0.0)
    assert np.allclose(ops.prox(Y, r, 1.0), expect, atol=1e-14)


def test_l1_ball_projection_matches_bisection():
    Y, r = _rand(100, 9, 5, scale=2.0)
    P = ops.project(Y, r, np.inf)
    for l in range(Y.shape[0]):
        assert np.allclose(P[l], proj_l1_bisection(Y[l], r[l]), atol=1e-12)


def test_l1_ball_projection_is_nearest_point():
    # no random feasible point is closer to y than the projection
    rng = np.random.default_rng(6)
    Y, r = _rand(20, 6, 6, scale=3.0)
    P = ops.project(Y, r, np.inf)
    for l in range(Y.shape[0]):
        dp = np.linalg.norm(Y[l] - P[l])
        for _ in range(200):
            u = rng.normal(size=6)
            u *= r[l] * rng.uniform() / np.abs(u).sum()
            assert np.linalg.norm(Y[l] - u) >= dp - 1e-12


def test_projection_zero_radius():
    Y, _ = _rand(10, 4, 7)
    r = np.zeros(10)
    for q in QS:
        assert np.all(ops.project(Y, r, q) == 0.0)


@pytest.mark.parametrize("q", QS)
def test_jacobian_matches_finite_differences(q):
    # at generic points (away from kinks) P = dPi/dY exactly
    Y, r = _rand(60, 5, 8, scale=1.5)
    rng = np.random.default_rng(9)
    V = rng.normal(size=Y.shape)
    h = 1e-7
    fd = (ops.project(Y + h * V, r, q) - ops.project(Y - h * V, r, q)) / (2 * h)
    JV = ops.jacobian_apply(Y, r, q, V)
    assert np.allclose(JV, fd, atol=1e-6)


@pytest.mark.parametrize("q", QS)
def test_newton_matrix_symmetric_psd(q):
    rng = np.random.default_rng(10)
    n, m, d = 8, 16, 3
    src = rng.integers(0, n, m)
    dst = (src + 1 + rng.integers(0, n - 1, m)) % n
    B = oracle.incidence(src, dst, n)
    Y, r = _rand(m, d, 11, scale=2.0)
    sigma = 3.0
    N = n * d
    M = np.zeros((N, N))
    for c in range(N):
        V = np.zeros((n, d))
        V.flat[c] = 1.0
        M[:, c] = (V + sigma * (B.T @ ops.jacobian_apply(Y, r, q, B @ V))).ravel()
    assert np.allclose(M, M.T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() >= 1.0 - 1e-10


@pytest.mark.parametrize("q", QS)
def test_weak_duality(q):
    rng = np.random.default_rng(12)
    n, m, d = 10, 25, 3
    src = rng.integers(0, n, m)
    dst = (src + 1 + rng.integers(0, n - 1, m)) % n
    B = oracle.incidence(src, dst, n)
    A = rng.normal(size=(n, d))
    r = rng.uniform(0.1, 1.0, m)
    for t in range(20):
        X = rng.normal(size=(n, d))
        U = ops.project(rng.normal(size=(m, d)) * 3, r, q)
        assert ops.primal_objective(X, A, B, r, q) >= ops.dual_objective(U, A, B) - 1e-12


def test_distance_bound_contains_the_solution():
    # the bound from the duality gap is never below the true distance to X*,
    # equals zero at the two-point closed form, and tightens as (X, U) do
    from oracle import operators as ops
    rng = np.random.default_rng(77)
    A = rng.normal(size=(30, 3))
    src, dst, w, *_ = oracle.knn_graph(A, 4, 0.5)
    B = oracle.incidence(src, dst, 30)
    for q in (1.0, 2.0, np.inf):
        Xs, Us, _, _ = oracle.ssnal(A, src, dst, w, 0.3, q, 1e-12)
        for eps in (1e-1, 1e-3, 1e-6):
            Xp = Xs + eps * rng.normal(size=Xs.shape)
            Up = Us + eps * rng.normal(size=Us.shape)
            bound, res = ops.distance_bound(Xp, Up, A, B, 0.3 * w, q)
            assert bound >= np.linalg.norm(Xp - Xs) * (1 - 1e-9), (q, eps)
        b0, _ = ops.distance_bound(Xs, Us, A, B, 0.3 * w, q)
        assert b0 <= 1e-5 * np.linalg.norm(Xs), q
    # two points, q = 2: X* and U* in closed form give a zero gap
    A2 = np.array([[0.0, 0.0], [3.0, 4.0]])
    B2 = oracle.incidence(np.array([0]), np.array([1]), 2)
    g, wl = 0.5, 1.0
    delta = A2[0] - A2[1]
    u = g * wl * delta / np.linalg.norm(delta)
    X2 = A2 - (B2.T @ u[None, :])
    b2, res2 = ops.distance_bound(X2, u[None, :], A2, B2, np.array([g * wl]), 2.0)
    allowance = np.sqrt(2e-13 * (1 + abs(res2["f_p"]) + abs(res2["f_d"])))
    assert b2 <= 1.01 * allowance and res2["kkt"] <= 1e-15
    assert abs(res2["f_p"] - res2["f_d"]) <= 1e-13 * abs(res2["f_p"])
