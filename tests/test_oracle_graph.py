"""Pins for the oracle's k-NN Gaussian weight graph.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import synthdata


def python_knn(A, k):
    """Pure-Python brute force: d^2 summed feature by feature, sorted by
    (d^2, index), self excluded."""
    n, d = A.shape
    out = []
    for i in range(n):
        cand = []
        for j in range(n):
            if j == i:
                continue
            s = 0.0
            for t in range(d):
                diff = float(A[i, t]) - float(A[j, t])
                s = s + diff * diff
            cand.append((s, j))
        cand.sort()
        out.append(cand[:k])
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_knn_matches_python_brute_force(seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(37, 5))
    A[7] = A[3]  # an exact duplicate (distance 0)
    idx, d2 = oracle.knn_brute(A, 6)
    ref = python_knn(A, 6)
    for i in range(A.shape[0]):
        assert [j for _, j in ref[i]] == idx[i].tolist()
        assert [s for s, _ in ref[i]] == d2[i].tolist()  # bit-exact


def test_knn_ties_break_by_index():
    # points on a line at integer spacing: equal distances on both sides
    A = np.arange(10, dtype=np.float64)[:, None]
    idx, d2 = oracle.knn_brute(A, 2)
    assert idx[5].tolist() == [4, 6]
    assert idx[0].tolist() == [1, 2]


def test_quantised_distances_are_exact_integers():
    # integer-valued data: every FP64 distance is an exact integer
    A, y, K = synthdata.images784(n_per=30, d=50, n_classes=3)
    Ki = K.astype(np.float64)
    idx, d2 = oracle.knn_brute(Ki, 10)
    exact = np.array([[int(((K[i].astype(np.int64) - K[j].astype(np.int64)) ** 2).sum())
                       for j in idx[i]] for i in range(K.shape[0])])
    assert np.array_equal(d2, exact.astype(np.float64))


def test_union_symmetrisation_and_weights():
    A, _ = synthdata.blobs2d(n_per=10)
    k = 4
    src, dst, w, phi, idx, d2 = oracle.knn_graph(A, k, phi=None)
    n = A.shape[0]
    pairs = set()
    for i in range(n):
        for j in idx[i]:
            pairs.add((min(i, int(j)), max(i, int(j))))
    assert sorted(pairs) == list(zip(src.tolist(), dst.tolist()))
    assert phi == 1.0 / float(np.median(d2))
    for l in range(src.size):
        i, j = int(src[l]), int(dst[l])
        dd = sum((A[i, t] - A[j, t]) ** 2 for t in range(A.shape[1]))
        assert math.isclose(w[l], math.exp(-phi * dd), rel_tol=1e-13)
    # fixed phi
    _, _, w2, phi2, _, _ = oracle.knn_graph(A, k, phi=0.5)
    assert phi2 == 0.5 and np.all(w2 > 0) and np.all(w2 <= 1)


def test_canonicalize_merges_and_drops():
    src = np.array([3, 1, 1, 2, 4, 0])
    dst = np.array([1, 3, 1, 0, 4, 2])
    w = np.array([0.5, 0.25, 9.0, 1.0, 2.0, 0.0])
    s, d, ww = oracle.canonicalize_edges(src, dst, w)
    assert s.tolist() == [0, 1] and d.tolist() == [2, 3]
    assert ww.tolist() == [1.0, 0.75]


def test_u8_knn_matches_python_brute_force():
    rng = np.random.default_rng(5)
    K = rng.integers(0, 4, size=(40, 6)).astype(np.uint8)  # many ties
    idx, D = oracle.knn_brute_u8(K, 5)
    for i in range(K.shape[0]):
        cand = sorted((int(((K[i].astype(int) - K[j].astype(int)) ** 2).sum()), j)
                      for j in range(K.shape[0]) if j != i)[:5]
        assert [j for _, j in cand] == idx[i].tolist()
        assert [dd for dd, _ in cand] == D[i].tolist()
    src, dst, w, phi, _, d2 = oracle.knn_graph_u8(K, 0.5, 5)
    assert np.all(d2 == D * 0.25)
