"""Vector-Jacobian product of the solution map X*(A, w, gamma) (oracle).

Test infrastructure only (see the package header).

q = 2 only.  At a solution whose cluster partition is locally constant
(every edge has a positive fusion margin), the points of cluster c share one
value v_c and the model reduces to the smooth problem
    F(v) = 1/2 sum_c sum_{i in c} ||v_c - a_i||^2
           + gamma sum_{inter-cluster l} w_l ||v_{c(i_l)} - v_{c(j_l)}||_2 .
Its stationarity condition, differentiated implicitly, gives the adjoint
system
    (diag(|c|) (x) I_d + B_c^T H B_c) lambda = g,   g_c = sum_{i in c} dL/dx_i,
    H_l = gamma w_l (I - ghat ghat^T) / ||delta_l||,  delta_l = x_i - x_j,
and then
    dL/da_i      = lambda_{c(i)},
    dL/dgamma    = - sum_inter w_l <(B_c lambda)_l, ghat_l>,
    dL/dlog w_l  = - gamma w_l <(B_c lambda)_l, ghat_l>   (0 inside a cluster).
This is the exact limit of (I + sigma B^T P B)^{-1} applied to the SSNAL
generalized Jacobian as sigma grows.

The reduced system is assembled as a sparse (K d) x (K d) matrix and solved
by a sparse direct solve for small K d, else by plain CG to 1e-14.

Parity: pinned by central finite differences of tight oracle solves and by
the closed forms at full fusion (dL/da_i = component mean of dL/dx) and at
gamma -> 0 (dL/dA = dL/dX), in tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .labels import cluster_labels, fusion_scale


def path_vjp(A, src, dst, w, gamma, X, dLdX, labels=None, direct_limit=60000):
    """Returns (dL/dA [n,d], dL/dlog w [m], dL/dgamma)."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n, d = A.shape
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    m = src.shape[0]
    if labels is None:
        labels, K = cluster_labels(X, src, dst, n, fusion_scale(A))
    labels = np.asarray(labels, dtype=np.int64)
    K = int(labels.max()) + 1 if n else 0
    size = np.bincount(labels, minlength=K).astype(np.float64)
    g = np.zeros((K, d))
    np.add.at(g, labels, dLdX)
    ci = labels[src]
    cj = labels[dst]
    inter = ci != cj
    li = np.nonzero(inter)[0]
    delta = X[src[li]] - X[dst[li]]
    nd = np.sqrt((delta * delta).sum(axis=1))
    gh = delta / nd[:, None]
    coef = gamma * w[li] / nd
    # assemble H_F = diag(|c|) (x) I + sum_l (e_ci - e_cj)(e_ci - e_cj)^T (x) H_l
    rows, cols, vals = [], [], []
    kd = np.arange(K * d)
    rows.append(kd)
    cols.append(kd)
    vals.append(np.repeat(size, d))
    Il = np.eye(d)
    for t in range(li.size):
        Hl = coef[t] * (Il - np.outer(gh[t], gh[t]))
        a, b = ci[li[t]], cj[li[t]]
        for (p, s_), sign in (((a, a), 1.0), ((b, b), 1.0), ((a, b), -1.0), ((b, a), -1.0)):
            rr, cc = np.meshgrid(np.arange(d) + p * d, np.arange(d) + s_ * d, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(sign * Hl.ravel())
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(K * d, K * d))
    rhs = g.reshape(-1)
    if K * d <= direct_limit:
        lam = spla.spsolve(H.tocsc(), rhs)
    else:
        lam, info = spla.cg(H, rhs, rtol=1e-14, atol=0.0, maxiter=100000)
    lam = lam.reshape(K, d)
    dA = lam[labels]
    Bl = lam[ci[li]] - lam[cj[li]]
    proj = (Bl * gh).sum(axis=1)
    dlogw = np.zeros(m)
    dlogw[li] = -gamma * w[li] * proj
    dgamma = -float((w[li] * proj).sum())
    return dA, dlogw, dgamma
