"""Cluster labels from a solution X (oracle).

Test infrastructure only (see the package header).

Section 1 of the paper assigns a_i and a_j to one cluster iff x_i* = x_j*.
A computed X is only accurate to the solver tolerance, so the rule is read
numerically and over graph edges only (two points that are not linked by a
chain of edges coincide with probability zero):

* S = max_i ||a_i - abar||_2 is the spread of the data;
* edge l = (i, j) is fused iff ||x_i - x_j||_2 / (1 + S) <= 1e-5;
* clusters are the connected components of the fused edges, numbered by
  the rank of each component's smallest point index (so label 0 is the
  cluster of point 0).

The fusion margin of an edge at a (tight) primal-dual pair (X, U) is
max(s_l, t_l) with s_l the scaled gap above and t_l = 1 - ||u_l||_{q*}/r_l
the dual slack; a gamma is label-eligible when every margin exceeds 1e-4.

Parity: pinned by the two-point closed form (fused iff 2 gamma w >=
||a_1 - a_2||_{q*}) and by the full-fusion certificate; the numbering by a
hand-built graph with its label vector written out; the margins by the
two-point primal and dual solutions in closed form (primal gap below the
fusion threshold, dual slack above it, the dual norm where it differs from
the q-norm).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

FUSE_TOL = 1e-5
MARGIN_TOL = 1e-4


def fusion_scale(A):
    """S = max_i ||a_i - mean(a)||_2."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] == 0:
        return 0.0
    c = A - A.mean(axis=0)
    return float(np.sqrt((c * c).sum(axis=1)).max())


def fused_edges(X, src, dst, S, tol=FUSE_TOL):
    D = X[src] - X[dst]
    s = np.sqrt((D * D).sum(axis=1)) / (1.0 + S)
    return s <= tol, s


def canonical_components(n, src, dst, keep):
    """Connected components of the kept edges, labelled 0, 1, ... in order of
    each component's smallest vertex."""
    src = np.asarray(src)[keep]
    dst = np.asarray(dst)[keep]
    G = sp.coo_matrix((np.ones(src.shape[0]), (src, dst)), shape=(n, n))
    _, comp = connected_components(G, directed=False)
    # first occurrence order of comp ids when scanning vertices 0..n-1
    first = {}
    lab = np.empty(n, dtype=np.int32)
    for i in range(n):
        c = comp[i]
        if c not in first:
            first[c] = len(first)
        lab[i] = first[c]
    return lab, len(first)


def cluster_labels(X, src, dst, n, S, tol=FUSE_TOL):
    keep, _ = fused_edges(X, np.asarray(src), np.asarray(dst), S, tol)
    return canonical_components(n, src, dst, keep)


def fusion_margins(X, U, src, dst, w, gamma, q, S):
    """Per-edge margin max(s_l, t_l) (see module header)."""
    from .operators import row_norms, dual_exponent
    _, s = fused_edges(X, np.asarray(src), np.asarray(dst), S)
    r = gamma * np.asarray(w, dtype=np.float64)
    un = row_norms(U, dual_exponent(q))
    # at r = 0 the dual ball is {0}: no slack, the margin is the primal gap
    t = np.where(r > 0, 1.0 - un / np.where(r > 0, r, 1.0), 0.0)
    return np.maximum(s, t)
