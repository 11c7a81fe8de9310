"""Brute-force solvers for tiny (CCM) instances (oracle pins).

Test infrastructure only (see the package header).

Routes that share nothing with the SSNAL/ADMM code:

* ``dual_slsqp``: the dual min_{U in C} 1/2 ||A - B^T U||^2 handed to
  scipy's SLSQP with explicit constraints (q = 1: bounds |u| <= r;
  q = 2: r^2 - ||u_l||^2 >= 0; q = inf: u = u+ - u-, u+- >= 0,
  r - sum(u+ + u-) >= 0), X = A - B^T U.
* ``primal_value``: the (CCM) objective evaluated edge by edge in a
  Python loop, used to confirm that a candidate X is no worse than
  perturbations of it;
* ``proj_l1_bisection``: the l1-ball projection by bisection on the
  threshold.

Both use an explicit dense incidence matrix built in a Python loop.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def dense_incidence(src, dst, n):
    m = len(src)
    B = np.zeros((m, n))
    for l in range(m):
        B[l, int(src[l])] = 1.0
        B[l, int(dst[l])] = -1.0
    return B


def dual_slsqp(A, src, dst, w, gamma, q, maxiter=2000):
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    B = dense_incidence(src, dst, n)
    r = gamma * np.asarray(w, dtype=np.float64)
    a = A.reshape(-1)
    q = float(q)

    if np.isinf(q):
        # variables (u+, u-) >= 0, u = u+ - u-
        def unpack(v):
            return (v[: m * d] - v[m * d:]).reshape(m, d)

        def f(v):
            U = unpack(v)
            R = A - B.T @ U
            return 0.5 * float((R * R).sum())

        def grad(v):
            U = unpack(v)
            G = -(B @ (A - B.T @ U)).reshape(-1)
            return np.concatenate([G, -G])

        cons = [{"type": "ineq",
                 "fun": (lambda v, l=l: r[l] - v[l * d:(l + 1) * d].sum()
                         - v[m * d + l * d: m * d + (l + 1) * d].sum())}
                for l in range(m)]
        res = minimize(f, np.zeros(2 * m * d), jac=grad, method="SLSQP",
                       bounds=[(0.0, None)] * (2 * m * d), constraints=cons,
                       options=dict(maxiter=maxiter, ftol=1e-16))
        U = unpack(res.x)
    else:
        def f(u):
            U = u.reshape(m, d)
            R = A - B.T @ U
            return 0.5 * float((R * R).sum())

        def grad(u):
            U = u.reshape(m, d)
            return -(B @ (A - B.T @ U)).reshape(-1)

        if q == 1.0:
            bounds = [(-r[l], r[l]) for l in range(m) for _ in range(d)]
            res = minimize(f, np.zeros(m * d), jac=grad, method="SLSQP", bounds=bounds,
                           options=dict(maxiter=maxiter, ftol=1e-16))
        else:
            cons = [{"type": "ineq",
                     "fun": (lambda u, l=l: r[l] ** 2 - float((u[l * d:(l + 1) * d] ** 2).sum())),
                     "jac": (lambda u, l=l: _l2jac(u, l, d))}
                    for l in range(m)]
            res = minimize(f, np.zeros(m * d), jac=grad, method="SLSQP", constraints=cons,
                           options=dict(maxiter=maxiter, ftol=1e-16))
        U = res.x.reshape(m, d)
    X = (a - (B.T @ U).reshape(-1)).reshape(n, d)
    return X, U


def _l2jac(u, l, d):
    g = np.zeros_like(u)
    g[l * d:(l + 1) * d] = -2.0 * u[l * d:(l + 1) * d]
    return g


def primal_value(X, A, src, dst, w, gamma, q):
    """(CCM) objective by an explicit Python loop over edges."""
    X = np.asarray(X, dtype=np.float64)
    val = 0.5 * float(((X - A) ** 2).sum())
    for l in range(len(src)):
        z = X[int(src[l])] - X[int(dst[l])]
        if float(q) == 1.0:
            nz = float(np.abs(z).sum())
        elif float(q) == 2.0:
            nz = float(np.sqrt((z * z).sum()))
        else:
            nz = float(np.abs(z).max())
        val += gamma * float(w[l]) * nz
    return val


def proj_l1_bisection(y, r, iters=200):
    """Projection of one vector onto {||u||_1 <= r} by bisection on the
    threshold theta of sum (|y_k| - theta)_+ = r (independent of the
    sort-based oracle routine)."""
    y = np.asarray(y, dtype=np.float64)
    if np.abs(y).sum() <= r:
        return y.copy()
    lo, hi = 0.0, float(np.abs(y).max())
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if np.maximum(np.abs(y) - mid, 0.0).sum() > r:
            lo = mid
        else:
            hi = mid
    th = 0.5 * (lo + hi)
    return np.sign(y) * np.maximum(np.abs(y) - th, 0.0)
