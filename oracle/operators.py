"""Edge operators, projections, objectives and the KKT certificate (oracle).

Test infrastructure only (see the package header).

Notation, all following from the model (CCM) of Section 1 of the paper:

* A, X are n x d, row i is a_i / x_i.
* The edge set holds each unordered pair once, l = (i_l, j_l) with i_l < j_l
  and weight w_l > 0, matching the single sum over i < j in (CCM).
* B maps R^{n x d} -> R^{m x d}: (BX)_l = x_{i_l} - x_{j_l}; B^T is its
  adjoint.  With r_l = gamma w_l the model is
  min_X 1/2 ||X - A||_F^2 + p(BX),  p(Z) = sum_l r_l ||z_l||_q.
* q* is the dual exponent (1 <-> inf, 2 <-> 2) and C = {U : ||u_l||_{q*} <= r_l}.
  p is the support function of C, so prox_{t p}(y) = y - Pi_{tC}(y) (Moreau).
* The dual problem is max_{U in C} <A, B^T U> - 1/2 ||B^T U||^2 and the
  primal solution is X* = A - B^T U*.

Parity: pinned.  The projections are pinned by brute-force minimisation
and by the Moreau identity against a closed-form prox; the objectives and
KKT residuals by weak duality and by closed-form solutions (two points,
full fusion, gamma = 0) in tests/test_oracle_*.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def incidence(src, dst, n):
    """Sparse m x n matrix B with +1 at (l, i_l) and -1 at (l, j_l)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    m = src.shape[0]
    rows = np.concatenate([np.arange(m), np.arange(m)])
    cols = np.concatenate([src, dst])
    vals = np.concatenate([np.ones(m), -np.ones(m)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m, n))


def dual_exponent(q):
    q = float(q)
    if q == 1.0:
        return np.inf
    if q == 2.0:
        return 2.0
    if np.isinf(q):
        return 1.0
    raise ValueError("q must be 1, 2 or inf")


def row_norms(Z, q):
    """||z_l||_q for every row."""
    q = float(q)
    if q == 1.0:
        return np.abs(Z).sum(axis=1)
    if q == 2.0:
        return np.sqrt((Z * Z).sum(axis=1))
    if np.isinf(q):
        return np.abs(Z).max(axis=1) if Z.shape[1] else np.zeros(Z.shape[0])
    raise ValueError("q must be 1, 2 or inf")


def _proj_l2_ball(Y, r):
    nrm = np.sqrt((Y * Y).sum(axis=1))
    scale = np.ones_like(nrm)
    out = nrm > r
    scale[out] = r[out] / nrm[out]
    return Y * scale[:, None]


def _proj_box(Y, r):
    return np.clip(Y, -r[:, None], r[:, None])


def l1_threshold(Y, r):
    """For each row y with ||y||_1 > r, the theta >= 0 with
    sum_k (|y_k| - theta)_+ = r, by the sort-and-scan method (Held, Wolfe and
    Crowder 1974; Duchi et al. 2008).  Rows inside the ball get theta = 0
    (projection is the identity); rows with r = 0 get theta = max |y_k|.
    Returns (theta [m], outside mask [m])."""
    a = np.abs(Y)
    l1 = a.sum(axis=1)
    theta = np.zeros(Y.shape[0])
    outside = l1 > r
    idx = np.nonzero(outside)[0]
    if idx.size:
        s = -np.sort(-a[idx], axis=1)              # |y| sorted descending
        cs = np.cumsum(s, axis=1)
        j = np.arange(1, Y.shape[1] + 1, dtype=np.float64)
        rr = r[idx][:, None]
        cond = s - (cs - rr) / j > 0               # holds for j = 1..rho
        # rho = largest j where cond holds (cond is a prefix of trues)
        rho = cond.sum(axis=1)
        th = np.empty(idx.size)
        pos = rho > 0
        th[pos] = (cs[pos, rho[pos] - 1] - r[idx][pos]) / rho[pos]
        th[~pos] = s[~pos, 0]                      # r = 0: ball is {0}
        theta[idx] = th
    return theta, outside


def _proj_l1_ball(Y, r):
    theta, outside = l1_threshold(Y, r)
    out = Y.copy()
    if outside.any():
        Yo = Y[outside]
        out[outside] = np.sign(Yo) * np.maximum(np.abs(Yo) - theta[outside][:, None], 0.0)
    return out


def project(Y, r, q):
    """Row-wise Euclidean projection onto C = {||u_l||_{q*} <= r_l}.
    q = 2: l2 ball; q = 1: box [-r, r]; q = inf: l1 ball."""
    r = np.asarray(r, dtype=np.float64)
    q = float(q)
    if q == 2.0:
        return _proj_l2_ball(Y, r)
    if q == 1.0:
        return _proj_box(Y, r)
    if np.isinf(q):
        return _proj_l1_ball(Y, r)
    raise ValueError("q must be 1, 2 or inf")


def prox(Y, t_r, q):
    """prox of sum_l t_r[l] ||.||_q row-wise, by the Moreau identity."""
    return Y - project(Y, t_r, q)


def jacobian_apply(Y, r, q, V):
    """Apply an element P of the generalized Jacobian of Pi_C at Y to V,
    row by row.  On the ball boundary the identity branch is taken.

    q = 2: I inside, (r/||y||)(I - yhat yhat^T) outside;
    q = 1: diag(1[|y_k| <= r]);
    q = inf: I inside, diag(1_S) - s_S s_S^T / |S| outside, with
             S = {k : |y_k| > theta}, s = sign(y)."""
    r = np.asarray(r, dtype=np.float64)
    q = float(q)
    if q == 2.0:
        nrm = np.sqrt((Y * Y).sum(axis=1))
        out = V.copy()
        o = nrm > r
        if o.any():
            yh = Y[o] / nrm[o][:, None]
            c = (yh * V[o]).sum(axis=1)
            out[o] = (r[o] / nrm[o])[:, None] * (V[o] - yh * c[:, None])
        return out
    if q == 1.0:
        return V * (np.abs(Y) <= r[:, None])
    if np.isinf(q):
        theta, outside = l1_threshold(Y, r)
        out = V.copy()
        if outside.any():
            Yo, Vo = Y[outside], V[outside]
            S = np.abs(Yo) > theta[outside][:, None]
            s = np.sign(Yo) * S
            cnt = S.sum(axis=1)
            c = (s * Vo).sum(axis=1)
            res = Vo * S
            nz = cnt > 0
            res[nz] -= s[nz] * (c[nz] / cnt[nz])[:, None]
            out[outside] = res
        return out
    raise ValueError("q must be 1, 2 or inf")


def primal_objective(X, A, B, r, q):
    """f_p(X) = 1/2 ||X - A||^2 + sum_l r_l ||(BX)_l||_q."""
    D = X - A
    return 0.5 * float((D * D).sum()) + float((r * row_norms(B @ X, q)).sum())


def dual_objective(U, A, B):
    """f_d(U) = <A, B^T U> - 1/2 ||B^T U||^2 (valid as a bound for U in C)."""
    BtU = B.T @ U
    return float((A * BtU).sum()) - 0.5 * float((BtU * BtU).sum())


def kkt_residuals(X, U, A, B, r, q):
    """Relative KKT residuals and duality gap of (X, U).

    R_D = ||X - A + B^T U|| / (1 + ||A||)
    R_C = ||Pi_C(BX + U) - U|| / (1 + ||BX|| + ||U||)   (zero iff U in dp(BX))
    R_U = ||U - Pi_C(U)|| / (1 + ||U||)
    eta = |f_p(X) - f_d(Pi_C U)| / (1 + |f_p| + |f_d|)  (Section 4)
    Returns dict with R_D, R_C, R_U, kkt = max of the three, eta, f_p, f_d."""
    BX = B @ X
    nA = np.linalg.norm(A)
    nBX = np.linalg.norm(BX)
    nU = np.linalg.norm(U)
    RD = np.linalg.norm(X - A + B.T @ U) / (1.0 + nA)
    RC = np.linalg.norm(project(BX + U, r, q) - U) / (1.0 + nBX + nU)
    Uf = project(U, r, q)
    RU = np.linalg.norm(U - Uf) / (1.0 + nU)
    D = X - A
    fp = 0.5 * float((D * D).sum()) + float((r * row_norms(BX, q)).sum())
    fd = dual_objective(Uf, A, B)
    eta = abs(fp - fd) / (1.0 + abs(fp) + abs(fd))
    return dict(R_D=RD, R_C=RC, R_U=RU, kkt=max(RD, RC, RU), eta=eta, f_p=fp, f_d=fd)


def distance_bound(X, U, A, B, r, q):
    """Upper bound on ||X - X*||_F for the unique solution X* of (CCM).

    (CCM) is 1-strongly convex in X, so f_p(X) - f_p(X*) >= 1/2 ||X - X*||^2,
    and weak duality gives f_p(X*) >= f_d(Pi_C U) for any U; hence
    ||X - X*||^2 <= 2 (f_p(X) - f_d(Pi_C U)).  The gap is taken with a
    rounding allowance of 1e-13 (1 + |f_p| + |f_d|) for the two sums.
    Returns (bound, kkt_residuals(X, U, ...))."""
    res = kkt_residuals(X, U, A, B, r, q)
    fp, fd = res["f_p"], res["f_d"]
    gap = max(fp - fd, 0.0) + 1e-13 * (1.0 + abs(fp) + abs(fd))
    return float(np.sqrt(2.0 * gap)), res

