"""Pins for the oracle's cluster rule: the canonical label numbering and the
per-edge fusion margins that decide where labels are compared bit-exactly.
CPU only.

The margins are checked against the two-point problem, whose primal and
dual solutions are known in closed form: with delta = a_1 - a_2 and
t = 2 gamma w, x_1 - x_2 = prox_{t ||.||_q}(delta) and the edge's dual value
is u = (delta - (x_1 - x_2)) / 2.  Below the fusion threshold
(||delta||_{q*} > t) u lies on its ball boundary, so the dual slack is 0
and the margin is the primal gap s = ||x_1 - x_2||_2 / (1 + S); above it
x_1 = x_2, u = delta / 2 and the margin is the slack
1 - ||delta||_{q*} / t.
"""
import numpy as np
import pytest

import oracle
from oracle.brute import proj_l1_bisection

QS = [1.0, 2.0, np.inf]


def dual_norm(v, q):
    """||v||_{q*} written out per q (q* = inf for q = 1, 2 for 2, 1 for inf)."""
    if q == 1.0:
        return float(np.max(np.abs(v)))
    if q == 2.0:
        return float(np.sqrt(np.sum(v * v)))
    return float(np.sum(np.abs(v)))


def prox_textbook(delta, t, q):
    if q == 2.0:
        nd = np.sqrt(np.sum(delta * delta))
        return delta * max(0.0, 1.0 - t / nd)
    if q == 1.0:
        return np.sign(delta) * np.maximum(np.abs(delta) - t, 0.0)
    return delta - proj_l1_bisection(delta, t)


def two_point(delta_scale, gamma, w, q, seed):
    rng = np.random.default_rng(seed)
    # coordinates of clearly different magnitudes, so that the q-norm and
    # the dual norm of every vector below differ for q = 1 and q = inf
    a1 = np.array([0.3, -1.1, 2.0, 0.05]) * delta_scale + rng.normal(size=4) * 1e-3
    a2 = np.zeros(4)
    A = np.stack([a1, a2])
    delta = a1 - a2
    t = 2.0 * gamma * w
    diff = prox_textbook(delta, t, q)
    u = (delta - diff) / 2.0
    X = np.stack([a1 - u, a2 + u])
    return A, X, u[None, :], delta, diff


@pytest.mark.parametrize("q", QS)
def test_margin_below_fusion_threshold_is_primal_gap(q):
    gamma, w = 0.2, 0.9
    A, X, U, delta, diff = two_point(1.0, gamma, w, q, seed=1)
    assert dual_norm(delta, q) > 2 * gamma * w  # not fused
    S = oracle.fusion_scale(A)
    assert np.isclose(S, np.sqrt(np.sum(delta * delta)) / 2.0, rtol=1e-15)
    src, dst, wv = np.array([0]), np.array([1]), np.array([w])
    mg = oracle.fusion_margins(X, U, src, dst, wv, gamma, q, S)
    s = np.sqrt(np.sum(diff * diff)) / (1.0 + S)
    assert s > 1e-3
    # the dual value sits on its ball boundary: slack 0 up to rounding
    assert abs(dual_norm(U[0], q) / (gamma * w) - 1.0) <= 1e-12
    assert np.isclose(mg[0], s, rtol=1e-12, atol=0)


@pytest.mark.parametrize("q", QS)
def test_margin_above_fusion_threshold_is_dual_slack(q):
    gamma, w = 3.0, 0.9
    A, X, U, delta, diff = two_point(1.0, gamma, w, q, seed=2)
    assert dual_norm(delta, q) < 2 * gamma * w  # fused
    assert np.all(diff == 0.0)
    S = oracle.fusion_scale(A)
    src, dst, wv = np.array([0]), np.array([1]), np.array([w])
    mg = oracle.fusion_margins(X, U, src, dst, wv, gamma, q, S)
    expect = 1.0 - dual_norm(delta, q) / (2.0 * gamma * w)
    assert expect > 0.05
    assert np.isclose(mg[0], expect, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("q", [1.0, np.inf])
def test_margin_uses_the_dual_norm(q):
    """For q = 1 and inf the q-norm and the dual norm of u differ by a
    factor of several here; the slack must come from the dual norm."""
    gamma, w = 3.0, 0.9
    A, X, U, delta, _ = two_point(1.0, gamma, w, q, seed=3)
    S = oracle.fusion_scale(A)
    mg = oracle.fusion_margins(X, U, np.array([0]), np.array([1]), np.array([w]), gamma, q, S)
    u = U[0]
    qnorm = float(np.max(np.abs(u))) if q == np.inf else float(np.sum(np.abs(u)))
    wrong = 1.0 - qnorm / (gamma * w)
    right = 1.0 - dual_norm(u, q) / (gamma * w)
    assert abs(wrong - right) > 0.1
    assert np.isclose(mg[0], right, rtol=1e-12, atol=1e-15)


def test_margin_zero_radius_is_primal_gap():
    # gamma = 0: the dual ball is {0}, no slack; the margin is the gap
    A = np.array([[0.0, 0.0], [3.0, 4.0]])
    X = A.copy()
    U = np.zeros((1, 2))
    S = oracle.fusion_scale(A)  # 2.5
    mg = oracle.fusion_margins(X, U, np.array([0]), np.array([1]), np.array([1.0]), 0.0, 2.0, S)
    assert mg[0] == pytest.approx(5.0 / 3.5, rel=1e-15)


def test_label_numbering_by_smallest_point():
    """Hand-built graph: components {0, 5}, {1, 3, 6}, {2}, {4, 7}; the
    number of a cluster is the rank of its smallest point index."""
    n = 8
    # edges in scrambled order; fused ones join equal rows
    src = np.array([6, 0, 4, 1, 2, 3, 5, 2])
    dst = np.array([3, 5, 7, 3, 7, 4, 6, 1])
    X = np.zeros((n, 2))
    X[[0, 5]] = [1.0, 1.0]
    X[[1, 3, 6]] = [-2.0, 0.5]
    X[2] = [4.0, 4.0]
    X[[4, 7]] = [0.0, -3.0]
    lab, nc = oracle.cluster_labels(X, src, dst, n, S=1.0)
    assert nc == 4
    assert lab.tolist() == [0, 1, 2, 1, 3, 0, 1, 3]


def test_label_chain_and_tolerance_edge():
    """Fusion is transitive along chains of fused edges (1-2 and 2-3 fused,
    1-3 not an edge), and the threshold is inclusive:
    ||x_i - x_j|| / (1 + S) <= 1e-5."""
    n = 5
    S = 3.0
    tol_gap = 1e-5 * (1.0 + S)
    X = np.zeros((n, 1))
    X[0, 0] = 10.0
    X[1, 0] = 0.0
    X[2, 0] = 0.5 * tol_gap
    X[3, 0] = 1.0 * tol_gap       # 2-3 gap 0.5 tol, 1-3 gap 1.0 tol (no edge)
    X[4, 0] = 1.0 * tol_gap + 2.0 * tol_gap  # 3-4 gap 2 tol: cut; 0-4 far apart
    src = np.array([1, 2, 3, 0])
    dst = np.array([2, 3, 4, 4])
    lab, nc = oracle.cluster_labels(X, src, dst, n, S=S)
    assert lab.tolist() == [0, 1, 1, 1, 2]
    assert nc == 3
    # a gap of exactly the threshold is fused; just above it is not
    Y = np.array([[0.0], [4e-5]])
    assert oracle.cluster_labels(Y, np.array([0]), np.array([1]), 2, S=3.0)[1] == 1
    Y[1, 0] = 4e-5 * (1 + 1e-9)
    assert oracle.cluster_labels(Y, np.array([0]), np.array([1]), 2, S=3.0)[1] == 2


def test_isolated_points_are_own_clusters():
    X = np.zeros((4, 3))
    lab, nc = oracle.cluster_labels(X, np.array([2], np.int64), np.array([3], np.int64), 4, S=0.0)
    assert lab.tolist() == [0, 1, 2, 2] and nc == 3
