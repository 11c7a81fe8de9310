"""ADMM, SSNAL and fast AMA for the convex clustering model (oracle).

Test infrastructure only (see the package header).

The paper names the three solvers (Section 1, Table 3: ADMM and fast AMA of
Chi and Lange 2015; SSNAL of Yuan, Sun and Toh 2018) but prints none of
their steps, so each one here is written from the algorithm's definition
applied to (CCM); the heuristic parameters (sigma policy, forcing terms,
Armijo constants) are this implementation's choices and do not change the
unique minimiser X*.

SSNAL.  Augmented Lagrangian on  min 1/2||X-A||^2 + p(Z)  s.t.  BX = Z.
Eliminating Z leaves, for multiplier U and penalty sigma,
    phi(X) = 1/2||X-A||^2 + (||Y||^2 - ||Y - Pi_C(Y)||^2)/(2 sigma) - ||U||^2/(2 sigma)
           = 1/2||X-A||^2 + <BX, Pi_C(Y)> - ||Pi_C(Y) - U||^2/(2 sigma),
    Y = U + sigma BX,   grad phi = X - A + B^T Pi_C(Y),
whose generalized Hessian is I + sigma B^T P B with P in dPi_C(Y).  Each
outer step minimises phi by semismooth Newton (Jacobi-preconditioned CG for
the direction, Armijo backtracking), then sets U <- Pi_C(U + sigma BX).

ADMM.  Splitting of the same constrained form with multiplier L (Lambda):
    X <- (I + sigma B^T B)^{-1} (A + B^T(sigma Z - L)),
    Z <- prox_{p/sigma}(BX + L/sigma),   L <- L + tau sigma (BX - Z),
with residual balancing of sigma.

Fast AMA.  Accelerated projected gradient on the dual
min_{U in C} 1/2 ||A - B^T U||^2 with X = A - B^T U (FISTA with
gradient-based restart).

Stopping test for all three: the relative KKT residual of
operators.kkt_residuals (max of R_D, R_C, R_U) at most tol; the relative
duality gap eta of Section 4 is reported beside it.

Parity: pinned through tests/test_oracle_solvers.py (gamma = 0, two-point
closed forms for q = 1, 2, inf, full fusion certificate, centroid
invariance at every iterate, brute-force solves on tiny inputs, d = 1
textbook cases, equivariances, SSNAL/ADMM/AMA agreement).
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import (
    incidence,
    project,
    jacobian_apply,
    kkt_residuals,
    l1_threshold,
)
from .labels import cluster_labels, fusion_scale

SSNAL_DEFAULTS = dict(
    max_outer=300,
    max_newton=60,
    cg_maxit=500,
    sigma0=1.0,
    sigma_max=1e4,
    sigma_grow=2.0,
    rp_ratio=0.9,         # grow sigma only when R_P fell by less than 10%
    inner_floor=0.5,      # inner gradient target >= inner_floor * tol
    inner_rel=0.2,        # ... and >= inner_rel * R_P
    armijo=1e-4,
    ls_slack=1e-14,
    max_ls=40,
)

ADMM_DEFAULTS = dict(
    max_iter=20000,
    sigma0=1.0,
    tau=1.618,
    check_every=10,
    balance_every=50,
)

AMA_DEFAULTS = dict(max_iter=100000, check_every=10)

HPR_DEFAULTS = dict(
    max_iter=20000,
    sigma0=1.0,
    check_every=10,
    restart_sufficient=0.2,   # restart when the residual fell below 0.2 of the anchor's
    restart_necessary=0.8,    # ... or below 0.8 of it and rose since the last check
    restart_long=0.2,         # ... or the anchor is older than 0.2 of all iterations
)


def _diag_BtPB(Y, r, q, B_abs, d):
    """diag(B^T P B) as an n x d array: sum over incident edges of diag(P_l)."""
    q = float(q)
    m = Y.shape[0]
    if q == 2.0:
        nrm = np.sqrt((Y * Y).sum(axis=1))
        dg = np.ones((m, d))
        o = nrm > r
        if o.any():
            yh = Y[o] / nrm[o][:, None]
            dg[o] = (r[o] / nrm[o])[:, None] * (1.0 - yh * yh)
    elif q == 1.0:
        dg = (np.abs(Y) <= r[:, None]).astype(np.float64)
    else:
        theta, outside = l1_threshold(Y, r)
        dg = np.ones((m, d))
        if outside.any():
            S = np.abs(Y[outside]) > theta[outside][:, None]
            cnt = S.sum(axis=1)
            inv = np.where(cnt > 0, 1.0 / np.maximum(cnt, 1), 0.0)
            dg[outside] = S * (1.0 - inv[:, None])
    return B_abs.T @ dg


def _pcg(apply_A, b, diag, rtol, maxit):
    """Plain Jacobi-preconditioned conjugate gradient from x0 = 0.
    Stops when ||r|| <= rtol ||b||.  Returns (x, iterations)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0
    z = r / diag
    p = z.copy()
    rz = float((r * z).sum())
    it = 0
    for it in range(1, maxit + 1):
        Ap = apply_A(p)
        pAp = float((p * Ap).sum())
        if pAp <= 0.0:
            break
        alpha = rz / pAp
        x += alpha * p
        r -= alpha * Ap
        if np.linalg.norm(r) <= rtol * nb:
            break
        z = r / diag
        rz_new = float((r * z).sum())
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it


def ssnal_evaluate(Xc, Uc, s, A, B, Bt, r, q, nA):
    """SSNAL merit function at X for multiplier Uc and penalty s: the edge
    pass Y = U + s BX, Pi = Pi_C(Y), the gradient G = X - A + B^T Pi, phi,
    the gradient norm gn = ||G|| / (1 + ||A||) and the primal residual rp."""
    BX = B @ Xc
    Y = Uc + s * BX
    Pi = project(Y, r, q)
    G = Xc - A + Bt @ Pi
    Dx = Xc - A
    # with ||Y||^2 - ||Y - Pi||^2 = 2<Y, Pi> - ||Pi||^2 and Y = U + sigma BX,
    # phi = 1/2||X - A||^2 + <BX, Pi> - ||Pi - U||^2/(2 sigma): the same
    # value without two large terms that cancel
    phi = (0.5 * float((Dx * Dx).sum()) + float((BX * Pi).sum())
           - float(((Pi - Uc) ** 2).sum()) / (2.0 * s))
    gn = np.linalg.norm(G) / (1.0 + nA)
    rp = np.linalg.norm(Pi - Uc) / (s * (1.0 + np.linalg.norm(BX) + np.linalg.norm(Pi)))
    return dict(Y=Y, Pi=Pi, G=G, phi=phi, gn=gn, rp=rp)


def ssnal_hessian_apply(V, Y, s, B, Bt, r, q):
    """The SSNAL Newton matrix applied to V: V + s B^T P B V, P in dPi_C(Y)."""
    return V + s * (Bt @ jacobian_apply(Y, r, q, B @ V))


def ssnal(A, src, dst, w, gamma, q, tol=1e-6, X0=None, U0=None, sigma=None,
          opts=None, callback=None):
    """Solve (CCM) at one gamma by SSNAL.  Returns (X, U, sigma, info)."""
    o = dict(SSNAL_DEFAULTS)
    if opts:
        o.update(opts)
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    B = incidence(src, dst, n)
    Bt = B.T.tocsr()
    B_abs = abs(B)
    r = float(gamma) * np.asarray(w, dtype=np.float64)
    sig = float(o["sigma0"] if sigma is None else sigma)
    info = dict(outer=0, newton=0, cg=0, linesearch=0)
    if gamma == 0.0 or m == 0:
        X = A.copy()
        U = np.zeros((m, d))
        info.update(kkt_residuals(X, U, A, B, r, q))
        return X, U, sig, info
    X = A.copy() if X0 is None else np.array(X0, dtype=np.float64)
    U = np.zeros((m, d)) if U0 is None else np.array(U0, dtype=np.float64)
    nA = np.linalg.norm(A)

    def evaluate(Xc, Uc, s):
        return ssnal_evaluate(Xc, Uc, s, A, B, Bt, r, q, nA)

    rp_prev = np.inf
    res = None
    for k in range(o["max_outer"]):
        info["outer"] += 1
        ev = evaluate(X, U, sig)
        for _ in range(o["max_newton"]):
            if ev["gn"] <= max(o["inner_floor"] * tol, o["inner_rel"] * ev["rp"]):
                break
            Y = ev["Y"]
            diag = 1.0 + sig * _diag_BtPB(Y, r, q, B_abs, d)

            def hess(V, Y=Y):
                return ssnal_hessian_apply(V, Y, sig, B, Bt, r, q)

            rtol = min(0.1, ev["gn"] ** 0.2)
            D, it = _pcg(hess, -ev["G"], diag, rtol, o["cg_maxit"])
            info["cg"] += it
            info["newton"] += 1
            slope = float((ev["G"] * D).sum())
            if not slope < 0.0:
                D = -ev["G"]
                slope = float((ev["G"] * D).sum())
            alpha = 1.0
            for _t in range(o["max_ls"]):
                info["linesearch"] += 1
                Xt = X + alpha * D
                evt = evaluate(Xt, U, sig)
                # Armijo test with a rounding allowance: near the solution the
                # decrease falls below the resolution of phi
                slack = o["ls_slack"] * (1.0 + abs(ev["phi"]))
                if evt["phi"] <= ev["phi"] + o["armijo"] * alpha * slope + slack:
                    break
                alpha *= 0.5
            X, ev = Xt, evt
            if callback is not None:
                callback(X)
        U = ev["Pi"]
        res = kkt_residuals(X, U, A, B, r, q)
        if res["kkt"] <= tol:
            break
        if k >= 1 and ev["rp"] > o["rp_ratio"] * rp_prev:
            sig = min(o["sigma_max"], o["sigma_grow"] * sig)
        rp_prev = ev["rp"]
    info.update(res)
    return X, U, sig, info


def admm(A, src, dst, w, gamma, q, tol=1e-6, X0=None, Z0=None, L0=None,
         sigma=None, opts=None, callback=None):
    """Solve (CCM) at one gamma by ADMM.  Returns (X, U, (Z, L, sigma), info)
    with U = Pi_C(L) the dual estimate used by the KKT test."""
    o = dict(ADMM_DEFAULTS)
    if opts:
        o.update(opts)
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    B = incidence(src, dst, n)
    Bt = B.T.tocsr()
    r = float(gamma) * np.asarray(w, dtype=np.float64)
    sig = float(o["sigma0"] if sigma is None else sigma)
    info = dict(iters=0)
    if gamma == 0.0 or m == 0:
        X = A.copy()
        U = np.zeros((m, d))
        info.update(kkt_residuals(X, U, A, B, r, q))
        return X, U, (np.zeros((m, d)), np.zeros((m, d)), sig), info
    X = A.copy() if X0 is None else np.array(X0, dtype=np.float64)
    Z = (B @ X) if Z0 is None else np.array(Z0, dtype=np.float64)
    L = np.zeros((m, d)) if L0 is None else np.array(L0, dtype=np.float64)
    Lap = (Bt @ B).tocsc()
    I = sp.identity(n, format="csc")
    lu = spla.splu((I + sig * Lap).tocsc())
    res = None
    for it in range(1, o["max_iter"] + 1):
        info["iters"] = it
        X = lu.solve(A + Bt @ (sig * Z - L))
        BX = B @ X
        Z_old = Z
        Pi = project(sig * BX + L, r, q)
        Z = BX + L / sig - Pi / sig
        L = L + o["tau"] * sig * (BX - Z)
        if callback is not None:
            callback(X)
        if it % o["check_every"] == 0:
            U = project(L, r, q)
            res = kkt_residuals(X, U, A, B, r, q)
            if res["kkt"] <= tol:
                break
        if it % o["balance_every"] == 0:
            rp = np.linalg.norm(BX - Z)
            rd = sig * np.linalg.norm(Bt @ (Z - Z_old))
            if rp > 10.0 * rd:
                sig *= 2.0
                lu = spla.splu((I + sig * Lap).tocsc())
            elif rd > 10.0 * rp:
                sig *= 0.5
                lu = spla.splu((I + sig * Lap).tocsc())
    U = project(L, r, q)
    if res is None or info["iters"] % o["check_every"] != 0:
        res = kkt_residuals(X, U, A, B, r, q)
    info.update(res)
    return X, U, (Z, L, sig), info


def hpr(A, src, dst, w, gamma, q, tol=1e-6, X0=None, Z0=None, L0=None,
        sigma=None, opts=None, callback=None):
    """Solve (CCM) at one gamma by the Halpern-Peaceman-Rachford method (the
    conclusion's future-work algorithm; the paper states no steps).

    The splitting is ADMM's, min f(X) + g(Z) s.t. BX = Z with
    f = 1/2 ||X - A||^2 and g(Z) = sum_l r_l ||z_l||_q.  One Peaceman-Rachford
    step T maps w = (Z, L) to (Zh, Lh):
        X  = (I + sigma B^T B)^{-1} (A + B^T (sigma Z - L)),
        H  = 2 B X - Z                        (reflection: relaxation 2),
        Lh = Pi_C(sigma H + L),   Zh = H + (L - Lh) / sigma
    (Zh is the prox of g / sigma at H + L / sigma by Moreau).  Halpern's
    iteration anchors it at w0:  w <- w0 / (k + 2) + (k + 1) / (k + 2) T(w).
    Every check_every iterations: stop when the relative KKT residual of
    (X, Lh) is <= tol; restart the anchor (w0 <- w, k <- 0) when the
    fixed-point residual R = (sigma ||Z - Zh||^2 + ||L - Lh||^2 / sigma)^(1/2)
    fell below 0.2 of its value at the anchor, or below 0.8 of it while
    rising, or when the anchor is older than 0.2 of the iterations so far.
    At a restart sigma becomes ||L - L0|| / ||Z - Z0|| (the movement since
    the anchor; it balances the two terms of the weighted norm), kept within
    a factor 10 of the old sigma.
    Returns (X, U, (Z, L, sigma), info) with U = Lh (already in C)."""
    o = dict(HPR_DEFAULTS)
    if opts:
        o.update(opts)
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    B = incidence(src, dst, n)
    Bt = B.T.tocsr()
    r = float(gamma) * np.asarray(w, dtype=np.float64)
    sig = float(o["sigma0"] if sigma is None else sigma)
    info = dict(iters=0, restarts=0)
    if gamma == 0.0 or m == 0:
        X = A.copy()
        U = np.zeros((m, d))
        info.update(kkt_residuals(X, U, A, B, r, q))
        return X, U, (np.zeros((m, d)), np.zeros((m, d)), sig), info
    X = A.copy() if X0 is None else np.array(X0, dtype=np.float64)
    Z = (B @ X) if Z0 is None else np.array(Z0, dtype=np.float64)
    L = np.zeros((m, d)) if L0 is None else np.array(L0, dtype=np.float64)
    Lap = (Bt @ B).tocsc()
    I = sp.identity(n, format="csc")
    lu = spla.splu((I + sig * Lap).tocsc())
    Za, La = Z.copy(), L.copy()      # anchor
    k = 0
    R_anchor = None
    R_prev = None
    res = None
    U = None
    for it in range(1, o["max_iter"] + 1):
        info["iters"] = it
        X = lu.solve(A + Bt @ (sig * Z - L))
        BX = B @ X
        H = 2.0 * BX - Z
        Lh = project(sig * H + L, r, q)
        Zh = H + (L - Lh) / sig
        dz2 = float(((Z - Zh) ** 2).sum())
        dl2 = float(((L - Lh) ** 2).sum())
        U = Lh
        a = 1.0 / (k + 2.0)
        Z = a * Za + (1.0 - a) * Zh
        L = a * La + (1.0 - a) * Lh
        k += 1
        if callback is not None:
            callback(X)
        if it % o["check_every"] == 0:
            res = kkt_residuals(X, U, A, B, r, q)
            if res["kkt"] <= tol:
                break
            R = np.sqrt(sig * dz2 + dl2 / sig)
            if R_anchor is None:
                R_anchor = R
            elif (R <= o["restart_sufficient"] * R_anchor
                  or (R <= o["restart_necessary"] * R_anchor and R_prev is not None
                      and R > R_prev)
                  or k >= o["restart_long"] * it):
                info["restarts"] += 1
                mz = np.linalg.norm(Z - Za)
                ml = np.linalg.norm(L - La)
                if mz > 0.0 and ml > 0.0:
                    sig = min(max(ml / mz, 0.1 * sig), 10.0 * sig)
                    lu = spla.splu((I + sig * Lap).tocsc())
                Za, La = Z.copy(), L.copy()
                k = 0
                R_anchor = np.sqrt(sig * dz2 + dl2 / sig)
                R_prev = None
                continue
            R_prev = R
    if res is None or info["iters"] % o["check_every"] != 0:
        res = kkt_residuals(X, U, A, B, r, q)
    info.update(res)
    return X, U, (Z, L, sig), info


def ama(A, src, dst, w, gamma, q, tol=1e-6, U0=None, opts=None):
    """Solve (CCM) at one gamma by fast AMA (accelerated dual projected
    gradient).  Returns (X, U, info)."""
    o = dict(AMA_DEFAULTS)
    if opts:
        o.update(opts)
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    B = incidence(src, dst, n)
    Bt = B.T.tocsr()
    r = float(gamma) * np.asarray(w, dtype=np.float64)
    info = dict(iters=0)
    if gamma == 0.0 or m == 0:
        X = A.copy()
        U = np.zeros((m, d))
        info.update(kkt_residuals(X, U, A, B, r, q))
        return X, U, info
    # Lipschitz constant of the dual gradient: lambda_max(B^T B) <= 2 max degree
    deg = np.bincount(np.concatenate([src, dst]), minlength=n)
    nu = 1.0 / (2.0 * deg.max())
    U = np.zeros((m, d)) if U0 is None else project(np.asarray(U0, float), r, q)
    V = U.copy()
    t = 1.0
    res = None
    for it in range(1, o["max_iter"] + 1):
        info["iters"] = it
        Xv = A - Bt @ V
        U_new = project(V + nu * (B @ Xv), r, q)
        # gradient restart: momentum is dropped when it points uphill
        if float(((V - U_new) * (U_new - U)).sum()) > 0.0:
            t = 1.0
            V = U_new.copy()
        else:
            t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
            V = U_new + ((t - 1.0) / t_new) * (U_new - U)
            t = t_new
        U = U_new
        if it % o["check_every"] == 0:
            X = A - Bt @ U
            res = kkt_residuals(X, U, A, B, r, q)
            if res["kkt"] <= tol:
                break
    X = A - Bt @ U
    res = kkt_residuals(X, U, A, B, r, q)
    info.update(res)
    return X, U, info


def solve_path(A, src, dst, w, gammas, q, tol=1e-6, method="ssnal", opts=None):
    """Warm-started path over gammas (in the given order).  Returns a dict of
    per-gamma lists: X, U, labels, n_clusters, kkt (dicts), info, seconds."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    m = len(src)
    S = fusion_scale(A)
    out = dict(X=[], U=[], labels=[], n_clusters=[], kkt=[], info=[], seconds=[])
    X = U = None
    sig = None
    Z = L = None
    for g in gammas:
        t0 = time.perf_counter()
        if method == "ssnal":
            # the penalty restarts at sigma0 for every gamma (X and U are warm)
            X, U, _, info = ssnal(A, src, dst, w, g, q, tol, X0=X, U0=U, sigma=None, opts=opts)
        elif method == "admm":
            X, U, (Z, L, sig), info = admm(A, src, dst, w, g, q, tol, X0=X, Z0=Z, L0=L,
                                           sigma=sig, opts=opts)
        elif method == "ama":
            X, U, info = ama(A, src, dst, w, g, q, tol, U0=U, opts=opts)
        elif method == "hpr":
            X, U, (Z, L, sig), info = hpr(A, src, dst, w, g, q, tol, X0=X, Z0=Z, L0=L,
                                          sigma=sig, opts=opts)
        else:
            raise ValueError(method)
        out["seconds"].append(time.perf_counter() - t0)
        lab, nc = cluster_labels(X, src, dst, n, S)
        out["X"].append(X.copy())
        out["U"].append(U.copy())
        out["labels"].append(lab)
        out["n_clusters"].append(nc)
        out["kkt"].append({k: info[k] for k in ("R_D", "R_C", "R_U", "kkt", "eta", "f_p", "f_d")})
        out["info"].append(info)
    return out
