"""k-nearest-neighbour Gaussian weight graph (oracle).

Test infrastructure only (see the package header).

The paper's Data Processor (Section 2.2) computes the weights w_ij from the
data; the model (Section 1) only asks w_ij = w_ji >= 0.  This oracle reads
that as: exact k nearest neighbours of each point by squared Euclidean
distance (the point itself excluded, ties broken by the lower index),
union-symmetrised (i ~ j iff j in kNN(i) or i in kNN(j)), with Gaussian
weights w = exp(-phi d^2), phi either given or 1 / median of the n k
directed neighbour distances (NumPy median: mean of the two middle values
for an even count).  Edges whose weight underflows to zero are dropped.

The squared distance is defined as the FP64 sum of the rounded squares
fl((a_ik - a_jk)^2) added in ascending k, each product and sum rounded
separately (no fused multiply-add).  This fixes every bit of d^2, so the
neighbour order (d^2, index) is a function of A alone; it is symmetric
because fl(a - b)^2 = fl(b - a)^2.  No expansion ||a||^2 + ||b||^2 - 2 a.b
is used, so there is no cancellation.

Parity: pinned by a pure-Python brute force on tiny inputs and by exact
integer distances on quantised data (tests/test_oracle_graph.py).
"""
from __future__ import annotations

import numpy as np


def sq_dists_rows(A, rows):
    """Squared distances from A[rows] to every row of A, summed in ascending
    feature order (see the module header)."""
    Ar = A[rows]
    acc = np.zeros((Ar.shape[0], A.shape[0]))
    for k in range(A.shape[1]):
        diff = Ar[:, k][:, None] - A[:, k][None, :]
        sq = diff * diff
        acc += sq
    return acc


def knn_brute(A, k, rows=None, block=64):
    """k nearest neighbours (self excluded, order (d^2, index)) of the given
    rows (all rows by default).  Returns (idx int32 [r, k], d2 [r, k])."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    kk = min(k, n - 1)
    idx = np.empty((rows.shape[0], kk), dtype=np.int32)
    d2 = np.empty((rows.shape[0], kk))
    for s in range(0, rows.shape[0], block):
        rr = rows[s:s + block]
        D = sq_dists_rows(A, rr)
        D[np.arange(rr.shape[0]), rr] = np.inf
        # stable sort keeps ascending index order among equal distances
        order = np.argsort(D, axis=1, kind="stable")[:, :kk]
        idx[s:s + block] = order
        d2[s:s + block] = np.take_along_axis(D, order, axis=1)
    return idx, d2


def canonicalize_edges(src, dst, w):
    """Order each pair as (min, max), drop self-loops and zero weights, merge
    duplicates by summing their weights, sort by (i, j)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    i = np.minimum(src, dst)
    j = np.maximum(src, dst)
    keep = (i != j) & (w > 0)
    i, j, w = i[keep], j[keep], w[keep]
    order = np.lexsort((j, i))
    i, j, w = i[order], j[order], w[order]
    if i.size == 0:
        return i.astype(np.int32), j.astype(np.int32), w
    new = np.ones(i.size, dtype=bool)
    new[1:] = (i[1:] != i[:-1]) | (j[1:] != j[:-1])
    grp = np.cumsum(new) - 1
    wsum = np.zeros(grp[-1] + 1)
    np.add.at(wsum, grp, w)
    return i[new].astype(np.int32), j[new].astype(np.int32), wsum


def knn_graph(A, k, phi=None):
    """Union-symmetrised k-NN graph with Gaussian weights.
    Returns (src, dst, w, phi_used, knn_idx, knn_d2)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    idx, d2 = knn_brute(A, k)
    if phi is None or phi <= 0:
        med = float(np.median(d2)) if d2.size else 0.0
        phi = 1.0 / med if med > 0 else 1.0
    ii = np.repeat(np.arange(n), idx.shape[1])
    jj = idx.reshape(-1).astype(np.int64)
    dd = d2.reshape(-1)
    a = np.minimum(ii, jj)
    b = np.maximum(ii, jj)
    key = a * n + b
    key_u, first = np.unique(key, return_index=True)
    src = (key_u // n).astype(np.int32)
    dst = (key_u % n).astype(np.int32)
    dist = dd[first]
    w = np.exp(-phi * dist)
    keep = w > 0
    return src[keep], dst[keep], w[keep], phi, idx, d2


def knn_brute_u8(K, k, rows=None, block=64):
    """Exact integer k-NN of integer codes K (squared distances summed in
    int64, no rounding), self excluded, order (D, index).
    Returns (idx int32 [r, k], D int64 [r, k])."""
    K = np.asarray(K).astype(np.int64)
    n = K.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    kk = min(k, n - 1)
    idx = np.empty((rows.shape[0], kk), dtype=np.int32)
    D = np.empty((rows.shape[0], kk), dtype=np.int64)
    for s in range(0, rows.shape[0], block):
        rr = rows[s:s + block]
        diff = K[rr][:, None, :] - K[None, :, :]
        Db = (diff * diff).sum(axis=2)
        Db[np.arange(rr.shape[0]), rr] = np.iinfo(np.int64).max
        order = np.argsort(Db, axis=1, kind="stable")[:, :kk]
        idx[s:s + block] = order
        D[s:s + block] = np.take_along_axis(Db, order, axis=1)
    return idx, D


def knn_graph_u8(K, scale, k, phi=None):
    """Graph of the points scale * K from exact integer distances:
    d^2 = float(D) * scale * scale, otherwise as knn_graph."""
    K = np.asarray(K)
    n = K.shape[0]
    idx, D = knn_brute_u8(K, k)
    d2 = D.astype(np.float64) * scale * scale
    if phi is None or phi <= 0:
        med = float(np.median(d2)) if d2.size else 0.0
        phi = 1.0 / med if med > 0 else 1.0
    ii = np.repeat(np.arange(n), idx.shape[1])
    jj = idx.reshape(-1).astype(np.int64)
    a = np.minimum(ii, jj)
    b = np.maximum(ii, jj)
    key = a * n + b
    key_u, first = np.unique(key, return_index=True)
    src = (key_u // n).astype(np.int32)
    dst = (key_u % n).astype(np.int32)
    w = np.exp(-phi * d2.reshape(-1)[first])
    keep = w > 0
    return src[keep], dst[keep], w[keep], phi, idx, d2
