"""Pins for the oracle's implicit-differentiation adjoint (q = 2).  CPU only."""
import numpy as np
import pytest

import oracle
import synthdata

TIGHT = 1e-13


def _problem(n_per=6, seed=1005, d=3):
    A, _ = synthdata.mixture64(seed=seed, n_per=n_per, d=d, n_blobs=3)
    A = A / 3.0
    src, dst, w, *_ = oracle.knn_graph(A, 4, phi=None)
    return A, src, dst, w


def _loss(X, T):
    return float(((X - T) ** 2).sum())


def _solve(A, src, dst, w, g):
    X, U, _, info = oracle.ssnal(A, src, dst, w, g, 2.0, TIGHT)
    assert info["kkt"] <= 1e-12
    return X


def test_vjp_matches_central_differences():
    A, src, dst, w = _problem()
    rng = np.random.default_rng(7)
    T = rng.normal(size=A.shape)
    g = 0.1  # 16 clusters of 18 points, every fusion margin above 1e-2
    X = _solve(A, src, dst, w, g)
    S = oracle.fusion_scale(A)
    lab0, K = oracle.cluster_labels(X, src, dst, A.shape[0], S)
    assert 1 < K < A.shape[0]  # a genuinely partial fusion
    dA, dlogw, dg = oracle.path_vjp(A, src, dst, w, g, X, 2 * (X - T), labels=lab0)
    h = 1e-6
    checked = 0
    # a few random directions in A, log w and gamma
    for t in range(4):
        V = rng.normal(size=A.shape)
        Xp = _solve(A + h * V, src, dst, w, g)
        Xm = _solve(A - h * V, src, dst, w, g)
        lp, _ = oracle.cluster_labels(Xp, src, dst, A.shape[0], S)
        lm, _ = oracle.cluster_labels(Xm, src, dst, A.shape[0], S)
        if not (np.array_equal(lp, lab0) and np.array_equal(lm, lab0)):
            continue
        fd = (_loss(Xp, T) - _loss(Xm, T)) / (2 * h)
        assert abs(fd - float((dA * V).sum())) <= 1e-5 * (1 + abs(fd))
        checked += 1
    v = rng.normal(size=w.shape)
    Xp = _solve(A, src, dst, w * np.exp(h * v), g)
    Xm = _solve(A, src, dst, w * np.exp(-h * v), g)
    fd = (_loss(Xp, T) - _loss(Xm, T)) / (2 * h)
    assert abs(fd - float((dlogw * v).sum())) <= 1e-5 * (1 + abs(fd))
    Xp = _solve(A, src, dst, w, g + h)
    Xm = _solve(A, src, dst, w, g - h)
    fd = (_loss(Xp, T) - _loss(Xm, T)) / (2 * h)
    assert abs(fd - dg) <= 1e-5 * (1 + abs(fd))
    assert checked >= 2


def test_vjp_full_fusion_is_component_mean():
    A, src, dst, w = _problem(n_per=5)
    g = 50.0
    X = _solve(A, src, dst, w, g)
    rng = np.random.default_rng(8)
    G = rng.normal(size=A.shape)
    dA, dlogw, dg = oracle.path_vjp(A, src, dst, w, g, X, G)
    lab, K = oracle.cluster_labels(X, src, dst, A.shape[0], oracle.fusion_scale(A))
    for c in range(K):
        assert np.allclose(dA[lab == c], G[lab == c].mean(0), atol=1e-12)
    assert np.all(dlogw == 0) and dg == 0.0


def test_vjp_small_gamma_is_identity():
    A, src, dst, w = _problem(n_per=5)
    X = _solve(A, src, dst, w, 1e-9)
    G = np.random.default_rng(9).normal(size=A.shape)
    dA, _, _ = oracle.path_vjp(A, src, dst, w, 1e-9, X, G)
    assert np.allclose(dA, G, atol=1e-6)
