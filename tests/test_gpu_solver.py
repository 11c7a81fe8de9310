"""Path solvers of libccm against the oracle (GPU)."""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import operators as ops
from gpu_util import need_gpu, dev, host, graph_dev, rel

pytestmark = pytest.mark.gpu

QS = [1.0, 2.0, np.inf]
METHODS = {"ssnal": 0, "admm": 1, "ama": 2, "hpr": 3}


def _opts(ccm, method, **kw):
    return ccm.ccm_default_options(method=METHODS[method], **kw)


def _certify(A, src, dst, w, g, q, X, U, tol):
    """Oracle KKT certificate of a GPU (X, U) pair."""
    B = oracle.incidence(src, dst, A.shape[0])
    res = ops.kkt_residuals(X, U, A, B, g * w, q)
    assert res["kkt"] <= tol * 1.0001, res
    return res


def _compare_path(A, src, dst, w, gammas, q, method, tol_gpu, tol_oracle=1e-10,
                  x_tol=1e-5, opts_kw=None):
    torch, ccm = need_gpu()
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), gammas, q, tol_gpu,
                             opts=_opts(ccm, method, **(opts_kw or {})), want_U=True)
    ref = oracle.solve_path(A, src, dst, w, gammas, q, tol_oracle, method="ssnal")
    S = oracle.fusion_scale(A)
    for t, g in enumerate(gammas):
        X = host(out["X"][t])
        U = host(out["U"][t])
        assert out["status"][t] == 0, (t, g, out["status"][t], out["kkt"][t])
        _certify(A, src, dst, w, g, q, X, U, tol_gpu)
        assert rel(X, ref["X"][t]) <= x_tol, (t, g, rel(X, ref["X"][t]))
        # labels: bit-exact when every edge has a clear fusion margin
        mg = oracle.fusion_margins(ref["X"][t], ref["U"][t], src, dst, w, g, q, S)
        if mg.min() > 1e-4:
            assert np.array_equal(host(out["labels"][t]), ref["labels"][t]), (t, g)
            assert out["n_clusters"][t] == ref["n_clusters"][t]
    return out, ref


@pytest.mark.parametrize("method", ["ssnal", "admm", "hpr"])
def test_blobs2d_path(method):
    A, _ = synthdata.blobs2d()
    src, dst, w, *_ = oracle.knn_graph(A, 10, 0.5)
    gammas = synthdata.gamma_grid(-3, 1, 10)
    _compare_path(A, src, dst, w, gammas, 2.0, method, 1e-6, x_tol=1e-5)


@pytest.mark.parametrize("q", QS)
def test_small_path_all_q(q):
    A, _ = synthdata.mixture64(n_per=40, d=8, n_blobs=4)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    gammas = synthdata.gamma_grid(-2, 1, 6)
    _compare_path(A, src, dst, w, gammas, q, "ssnal", 1e-8, x_tol=1e-6)


@pytest.mark.parametrize("q", QS)
def test_hpr_small_all_q(q):
    A, _ = synthdata.mixture64(n_per=30, d=5, n_blobs=4, seed=1401)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    gammas = synthdata.gamma_grid(-2, 1, 5)
    _compare_path(A, src, dst, w, gammas, q, "hpr", 1e-8, x_tol=1e-6)


@pytest.mark.parametrize("q", QS)
def test_ama_small(q):
    A, _ = synthdata.blobs2d(n_per=15)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    gammas = synthdata.gamma_grid(-2, 0.5, 4)
    _compare_path(A, src, dst, w, gammas, q, "ama", 1e-7, x_tol=1e-5)


@pytest.mark.parametrize("d", [3, 64, 130])
def test_ragged_dims(d):
    A, _ = synthdata.mixture64(n_per=30, d=d, n_blobs=5, seed=7 + d)
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    gammas = [0.0, 0.05, 0.5, 5.0]
    _compare_path(A, src, dst, w, gammas, 2.0, "ssnal", 1e-8, x_tol=1e-6)


def test_gamma_zero_and_no_edges():
    torch, ccm = need_gpu()
    A = np.random.default_rng(0).normal(size=(20, 3))
    out = ccm.ccm_solve_path(dev(A), dev(np.zeros(0, np.int32)), dev(np.zeros(0, np.int32)),
                             dev(np.zeros(0)), [0.0, 1.0], 2.0, 1e-6)
    for t in range(2):
        assert np.array_equal(host(out["X"][t]), A)
        assert out["n_clusters"][t] == 20
        assert np.array_equal(host(out["labels"][t]), np.arange(20))


def test_noncanonical_edges_are_merged():
    torch, ccm = need_gpu()
    A, _ = synthdata.blobs2d(n_per=10)
    src, dst, w, *_ = oracle.knn_graph(A, 4, 0.5)
    # reversed duplicates with split weights, plus a self loop and a zero weight
    s2 = np.concatenate([dst, src, [3], [1]]).astype(np.int32)
    d2 = np.concatenate([src, dst, [3], [2]]).astype(np.int32)
    w2 = np.concatenate([0.25 * w, 0.75 * w, [1.0], [0.0]])
    g = [0.1, 0.4]
    out = ccm.ccm_solve_path(dev(A), *graph_dev(s2, d2, w2), g, 2.0, 1e-9)
    ref = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-9)
    for t in range(2):
        assert rel(host(out["X"][t]), host(ref["X"][t])) <= 1e-7


def test_deterministic():
    torch, ccm = need_gpu()
    A, _ = synthdata.mixture64(n_per=100, d=16, n_blobs=5)
    src, dst, w, *_ = oracle.knn_graph(A, 8, None)
    g = synthdata.gamma_grid(-2, 1, 5)
    a = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-7)
    b = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-7)
    assert torch.equal(a["X"], b["X"])
    assert np.array_equal(a["kkt"], b["kkt"])


def test_invalid_arguments():
    torch, ccm = need_gpu()
    A = dev(np.zeros((5, 2)))
    s, d_, w = graph_dev([0, 1], [1, 2], [1.0, 1.0])
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [0.1], 3.0, 1e-6)
    assert e.value.status == 2
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [-0.1], 2.0, 1e-6)
    assert e.value.status == 1
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, s, d_, w, [0.1], 2.0, 0.0)
    assert e.value.status == 1
    bad_s, bad_d, bad_w = graph_dev([0, 7], [1, 2], [1.0, 1.0])
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(A, bad_s, bad_d, bad_w, [0.1], 2.0, 1e-6)
    assert e.value.status == 1
    s3, d3, w3 = graph_dev([0, 1], [1, 2], [1.0, -1.0])
    with pytest.raises(ccm.CcmError):
        ccm.ccm_solve_path(A, s3, d3, w3, [0.1], 2.0, 1e-6)
    An = np.zeros((5, 2))
    An[2, 1] = np.nan
    with pytest.raises(ccm.CcmError):
        ccm.ccm_solve_path(dev(An), s, d_, w, [0.1], 2.0, 1e-6)
    An[2, 1] = -np.inf
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path(dev(An), s, d_, w, [0.1], 2.0, 1e-6)
    assert e.value.status == 1


def test_nonfinite_points_rejected_anywhere_in_a_large_array():
    # the device finiteness pass strides over more values than its grid has
    # threads: a bad value in the last row is still found
    torch, ccm = need_gpu()
    n, d = 40000, 64
    A = np.random.default_rng(3).normal(size=(n, d))
    for bad in (np.nan, np.inf):
        A2 = A.copy()
        A2[-1, -1] = bad
        with pytest.raises(ccm.CcmError) as e:
            ccm.ccm_build_knn_graph(dev(A2), 5, 0.0)
        assert e.value.status == 1
    s, d_, w, _ = ccm.ccm_build_knn_graph(dev(A), 5, 0.0)
    assert s.numel() >= n * 5 // 2


def test_release_workspace_between_solves_keeps_results():
    torch, ccm = need_gpu()
    A, _ = synthdata.blobs2d(n_per=30)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    g = [0.05, 0.3]
    one = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-8)
    ccm.ccm_release_workspace()
    two = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), g, 2.0, 1e-8)
    assert np.array_equal(host(one["X"]), host(two["X"]))
    ccm.ccm_release_workspace()


def test_max_iter_status_and_time_budget():
    torch, ccm = need_gpu()
    A, _ = synthdata.blobs2d(n_per=20)
    src, dst, w, *_ = oracle.knn_graph(A, 6, 0.5)
    o = ccm.ccm_default_options(max_outer=1, max_newton=1)
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [0.3], 2.0, 1e-12, opts=o)
    assert out["status"][0] == 1
    assert np.all(np.isfinite(host(out["X"][0])))
    o = ccm.ccm_default_options(time_budget_s=1e-9)
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [0.3, 0.6], 2.0, 1e-12, opts=o)
    assert out["status"][0] == 2


def _adjoint_problem(n_per=40, d=4, seed=1005):
    A, _, T = synthdata.mixture32(seed=seed, n_per=n_per, d=d, n_blobs=4)
    A = A / 3.0
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    return A, src, dst, w, T


def test_vjp_matches_oracle_gradient():
    torch, ccm = need_gpu()
    A, src, dst, w, T = _adjoint_problem()
    n = A.shape[0]
    S = oracle.fusion_scale(A)
    # a gamma with partial fusion and clear margins
    for g in (0.08, 0.15, 0.3):
        Xo, Uo, _, info = oracle.ssnal(A, src, dst, w, g, 2.0, 1e-12)
        lab, K = oracle.cluster_labels(Xo, src, dst, n, S)
        mg = oracle.fusion_margins(Xo, Uo, src, dst, w, g, 2.0, S)
        if 1 < K < n and mg.min() > 1e-3:
            break
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [g], 2.0, 1e-11)
    X = out["X"][0]
    assert np.array_equal(host(out["labels"][0]), lab)
    G = 2 * (host(X) - T)
    dA, dlw, dg, it = ccm.ccm_path_vjp(dev(A), *graph_dev(src, dst, w), g, X, out["labels"][0],
                                       dev(G), tol=1e-13)
    rA, rlw, rg = oracle.path_vjp(A, src, dst, w, g, Xo, 2 * (Xo - T), labels=lab)
    assert rel(host(dA), rA) <= 1e-6
    assert rel(host(dlw), rlw) <= 1e-6
    assert abs(dg - rg) <= 1e-6 * (1 + abs(rg))


def test_vjp_clusters_larger_than_a_window():
    # four clusters of 320 points at d = 40: each cluster's membership list
    # is longer than a window (256 entries), so the cluster sums of the
    # adjoint go through the split-window path
    torch, ccm = need_gpu()
    A, _, T = synthdata.mixture32(seed=1007, n_per=320, d=40, n_blobs=4)
    A = A / 3.0
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    n = A.shape[0]
    g = 8.0
    Xo, Uo, _, _ = oracle.ssnal(A, src, dst, w, g, 2.0, 1e-12)
    lab, K = oracle.cluster_labels(Xo, src, dst, n, oracle.fusion_scale(A))
    assert K == 4 and np.bincount(lab).min() > 256
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [g], 2.0, 1e-11)
    X = out["X"][0]
    assert np.array_equal(host(out["labels"][0]), lab)
    dA, dlw, dg, _ = ccm.ccm_path_vjp(dev(A), *graph_dev(src, dst, w), g, X, out["labels"][0],
                                      dev(2 * (host(X) - T)), tol=1e-13)
    rA, rlw, rg = oracle.path_vjp(A, src, dst, w, g, Xo, 2 * (Xo - T), labels=lab)
    assert rel(host(dA), rA) <= 1e-6
    assert rel(host(dlw), rlw) <= 1e-6
    assert abs(dg - rg) <= 1e-6 * (1 + abs(rg))


def test_vjp_central_differences_on_gpu():
    torch, ccm = need_gpu()
    A, src, dst, w, T = _adjoint_problem(n_per=30, d=3, seed=77)
    g = 0.12
    sd = graph_dev(src, dst, w)

    def solve(Ah, wh, gh):
        o = ccm.ccm_solve_path(dev(Ah), sd[0], sd[1], dev(wh), [gh], 2.0, 1e-12)
        return host(o["X"][0]), host(o["labels"][0])

    X0, lab0 = solve(A, w, g)
    loss = lambda X: float(((X - T) ** 2).sum())
    out = ccm.ccm_solve_path(dev(A), *sd, [g], 2.0, 1e-12)
    dA, dlw, dg, _ = ccm.ccm_path_vjp(dev(A), *sd, g, out["X"][0], out["labels"][0],
                                      dev(2 * (X0 - T)), tol=1e-13)
    dA, dlw = host(dA), host(dlw)
    rng = np.random.default_rng(3)
    h = 1e-6
    checked = 0
    for _ in range(4):
        V = rng.normal(size=A.shape)
        Xp, lp = solve(A + h * V, w, g)
        Xm, lm = solve(A - h * V, w, g)
        if not (np.array_equal(lp, lab0) and np.array_equal(lm, lab0)):
            continue
        fd = (loss(Xp) - loss(Xm)) / (2 * h)
        assert abs(fd - float((dA * V).sum())) <= 1e-5 * (1 + abs(fd))
        checked += 1
    v = rng.normal(size=w.shape)
    Xp, _ = solve(A, w * np.exp(h * v), g)
    Xm, _ = solve(A, w * np.exp(-h * v), g)
    fd = (loss(Xp) - loss(Xm)) / (2 * h)
    assert abs(fd - float((dlw * v).sum())) <= 1e-5 * (1 + abs(fd))
    Xp, _ = solve(A, w, g + h)
    Xm, _ = solve(A, w, g - h)
    fd = (loss(Xp) - loss(Xm)) / (2 * h)
    assert abs(fd - dg) <= 1e-5 * (1 + abs(fd))
    assert checked >= 2


def test_ccmsolve_autograd():
    torch, ccm = need_gpu()
    A, src, dst, w, T = _adjoint_problem(n_per=20, d=3, seed=5)
    At = dev(A).requires_grad_(True)
    lw = dev(np.log(w)).requires_grad_(True)
    gam = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    s, d_, _ = graph_dev(src, dst, w)
    X = ccm.CCMSolve.apply(At, lw, gam, s, d_)
    L = ((X - dev(T)) ** 2).sum()
    L.backward()
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [0.1], 2.0, 1e-11)
    dA, dlw, dg, _ = ccm.ccm_path_vjp(dev(A), *graph_dev(src, dst, w), 0.1, out["X"][0],
                                      out["labels"][0], 2 * (out["X"][0] - dev(T)))
    assert torch.allclose(At.grad, dA, rtol=1e-8, atol=1e-10)
    assert torch.allclose(lw.grad, dlw, rtol=1e-8, atol=1e-10)
    assert abs(float(gam.grad) - dg) <= 1e-8 * (1 + abs(dg))


def _instances(count, seed, n_lo=30, n_hi=90, dims=(2, 3, 8), qs=(1.0, 2.0, np.inf)):
    insts = synthdata.instances(seed=seed, count=count, n_lo=n_lo, n_hi=n_hi, dims=dims,
                                blobs_lo=2, blobs_hi=4, qs=qs)
    out = []
    for it in insts:
        A = it["A"]
        src, dst, w, *_ = oracle.knn_graph(A, 5, None)
        out.append(dict(A=A, src=src, dst=dst, w=w, q=it["q"]))
    return out


def test_batched_matches_single_instance_solves():
    torch, ccm = need_gpu()
    insts = _instances(9, seed=21)
    gammas = synthdata.gamma_grid(-2, 0.5, 4)
    dev_insts = [dict(A=dev(i["A"]), src=dev(i["src"].astype(np.int32)),
                      dst=dev(i["dst"].astype(np.int32)), w=dev(i["w"]), q=i["q"]) for i in insts]
    res = ccm.ccm_solve_path_batched(dev_insts, gammas, 1e-8)
    for k, inst in enumerate(insts):
        ref = oracle.solve_path(inst["A"], inst["src"], inst["dst"], inst["w"], gammas,
                                inst["q"], 1e-10)
        B = oracle.incidence(inst["src"], inst["dst"], inst["A"].shape[0])
        S = oracle.fusion_scale(inst["A"])
        for t, g in enumerate(gammas):
            X = host(res[k]["X"][t])
            assert res[k]["status"][t] == 0, (k, t, res[k]["kkt"][t])
            assert res[k]["kkt"][t][:3].max() <= 1e-8
            assert rel(X, ref["X"][t]) <= 1e-6, (k, t)
            mg = oracle.fusion_margins(ref["X"][t], ref["U"][t], inst["src"], inst["dst"],
                                       inst["w"], g, inst["q"], S)
            if mg.min() > 1e-4:
                assert np.array_equal(host(res[k]["labels"][t]), ref["labels"][t])
                assert res[k]["n_clusters"][t] == ref["n_clusters"][t]


@pytest.mark.parametrize("q,method", [(1.0, "ssnal"), (2.0, "ssnal"), (np.inf, "ssnal"),
                                      (2.0, "admm")])
def test_path_with_a_hub_longer_than_a_window(q, method):
    # the fused edge pass + gradient (q = 1, 2), the scatter (q = inf) and the
    # Laplacian matvec of ADMM on a graph whose hub has more incidences than a
    # window holds
    rng = np.random.default_rng(1200)
    n, d = 700, 40  # rows of 40 values: windows of at most 256 incidences
    A = rng.normal(size=(n, d))
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    keys = {(int(a), int(b)): float(c) for a, b, c in zip(src, dst, w)}
    for j in rng.choice(np.arange(1, n), 400, replace=False):
        keys.setdefault((0, int(j)), float(rng.uniform(0.05, 0.3)))
    e = sorted(keys)
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    w = np.array([keys[k] for k in e])
    assert np.bincount(np.r_[src, dst], minlength=n).max() >= 400
    _compare_path(A, src, dst, w, [0.01, 0.05], q, method, 1e-7, x_tol=1e-5)


@pytest.mark.parametrize("q", QS)
def test_path_long_rows(q):
    # rows of 300 values: for q = 1, 2 the KKT terms come from the fused
    # edge pass of the next outer iteration (one launch)
    rng = np.random.default_rng(1300)
    n, d = 180, 300
    centres = rng.normal(size=(3, d)) * 2.0
    A = centres[rng.integers(0, 3, size=n)] + rng.normal(size=(n, d))
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    _compare_path(A, src, dst, w, [0.02, 0.2, 2.0], q, "ssnal", 1e-7, x_tol=1e-5)


def test_batched_groups_concurrent_and_reproducible():
    # the (q, d) groups run at once on streams of their own: results are the
    # same run to run and when the call is made on a side stream whose own
    # work produced the inputs just before
    torch, ccm = need_gpu()
    insts = _instances(12, seed=23)
    assert len({(i["q"], i["A"].shape[1]) for i in insts}) >= 5
    gammas = synthdata.gamma_grid(-2, 0.5, 3)
    dev_insts = [dict(A=dev(i["A"]), src=dev(i["src"].astype(np.int32)),
                      dst=dev(i["dst"].astype(np.int32)), w=dev(i["w"]), q=i["q"]) for i in insts]
    one = ccm.ccm_solve_path_batched(dev_insts, gammas, 1e-8)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        moved = [dict(x, A=x["A"] * 1.0) for x in dev_insts]
        two = ccm.ccm_solve_path_batched(moved, gammas, 1e-8, stream=side)
    side.synchronize()
    for a, b in zip(one, two):
        assert np.array_equal(host(a["X"]), host(b["X"]))
        assert np.array_equal(host(a["labels"]), host(b["labels"]))
        assert np.array_equal(np.asarray(a["status"]), np.asarray(b["status"]))
        assert np.all(np.asarray(a["status"]) == 0)


def test_batched_rejects_bad_descriptor():
    torch, ccm = need_gpu()
    insts = _instances(2, seed=22)
    d_insts = [dict(A=dev(i["A"]), src=dev(i["src"].astype(np.int32)),
                    dst=dev(i["dst"].astype(np.int32)), w=dev(i["w"]), q=i["q"]) for i in insts]
    bad = dict(d_insts[1])
    bad["dst"] = bad["dst"].clone()
    bad["dst"][0] = insts[1]["A"].shape[0] + 3  # outside the instance
    with pytest.raises(ccm.CcmError) as e:
        ccm.ccm_solve_path_batched([d_insts[0], bad], [0.1], 1e-6)
    assert e.value.status == 1


def test_qinf_tiny_weights_path():
    # k-NN Gaussian weights span many decades; q = inf radii reach 1e-22
    torch, ccm = need_gpu()
    insts = synthdata.instances(count=40)
    it = [i for i in insts if i["q"] == np.inf and i["d"] == 2][0]
    A = it["A"]  # n = 3156, weights down to 2e-35
    src, dst, w, *_ = oracle.knn_graph(A, 10, None)
    assert w.min() < 1e-30
    gammas = [1e-3, 1e-2]
    _compare_path(A, src, dst, w, gammas, np.inf, "ssnal", 1e-7, x_tol=1e-5)


def _with_tiny_weights(w):
    # Gaussian weights of far neighbours underflow: put subnormal, tiny and
    # zero weights on a share of the edges (gamma w then falls below the
    # radius at which 1/r stops being finite)
    w = w.copy()
    w[0::7] = 1e-310
    w[1::11] = 5e-324
    w[2::13] = 1e-200
    w[3::17] = 0.0
    return w


def _tiny_weight_graph(seed=1601):
    A, _ = synthdata.mixture64(n_per=60, d=2, n_blobs=5, seed=seed)
    src, dst, w, *_ = oracle.knn_graph(A, 8, None)
    return A, src, dst, _with_tiny_weights(w)


@pytest.mark.parametrize("q", [2.0, 1.0, np.inf])
def test_subnormal_and_tiny_weights(q):
    torch, ccm = need_gpu()
    A, src, dst, w = _tiny_weight_graph()
    # the library drops the zero-weight edges (U has a row per kept edge)
    keep = w > 0
    B = oracle.incidence(src[keep], dst[keep], A.shape[0])
    gammas = [1e-2, 0.2, 1.0]
    for method in (0, 1, 3):
        o = ccm.ccm_default_options(method=method)
        out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), gammas, q, 1e-8, opts=o,
                                 want_U=True)
        for t, g in enumerate(gammas):
            assert int(out["status"][t]) == 0, (method, t)
            X, U = host(out["X"][t]), host(out["U"][t])
            assert np.all(np.isfinite(X)) and np.all(np.isfinite(U))
            bound, res = oracle.operators.distance_bound(X, U, A, B, g * w[keep], q)
            assert res["kkt"] <= 1e-8 * 1.0001, (method, t, res)
            assert bound <= 1e-5 * np.linalg.norm(X), (method, t, bound)


def test_vjp_with_tiny_weights():
    torch, ccm = need_gpu()
    A, src, dst, w, T = _adjoint_problem(seed=1602)
    w = _with_tiny_weights(w)
    keep = w > 0  # the adjoint takes canonical edges (w > 0)
    src, dst, w = src[keep], dst[keep], w[keep]
    n = A.shape[0]
    S = oracle.fusion_scale(A)
    # (an edge of negligible weight has no dual slack; the labels do not
    # depend on its margin)
    big = w > 1e-100
    for g in (0.08, 0.15, 0.3):
        Xo, Uo, _, _ = oracle.ssnal(A, src, dst, w, g, 2.0, 1e-12)
        lab, K = oracle.cluster_labels(Xo, src, dst, n, S)
        mg = oracle.fusion_margins(Xo, Uo, src, dst, w, g, 2.0, S)
        if 1 < K < n and mg[big].min() > 1e-3:
            break
    assert 1 < K < n and mg[big].min() > 1e-3
    out = ccm.ccm_solve_path(dev(A), *graph_dev(src, dst, w), [g], 2.0, 1e-11)
    X = out["X"][0]
    assert np.array_equal(host(out["labels"][0]), lab)
    dA, dlw, dg, _ = ccm.ccm_path_vjp(dev(A), *graph_dev(src, dst, w), g, X, out["labels"][0],
                                      dev(2 * (host(X) - T)), tol=1e-13)
    rA, rlw, rg = oracle.path_vjp(A, src, dst, w, g, Xo, 2 * (Xo - T), labels=lab)
    assert np.all(np.isfinite(host(dA))) and np.all(np.isfinite(host(dlw)))
    assert rel(host(dA), rA) <= 1e-6
    assert rel(host(dlw), rlw) <= 1e-6
    assert abs(dg - rg) <= 1e-6 * (1 + abs(rg))


@pytest.mark.parametrize("q", [np.inf, 2.0])
def test_long_rows_with_a_hub(q):
    # rows of 300 values (q = inf takes the fused edge pass there) on a graph
    # whose hub has more incidences than a window holds (at most 256 here)
    rng = np.random.default_rng(1210)
    n, d = 320, 300
    A = rng.normal(size=(n, d)) + 3.0 * rng.normal(size=(3, d))[rng.integers(0, 3, size=n)]
    src, dst, w, *_ = oracle.knn_graph(A, 5, None)
    keys = {(int(a), int(b)): float(c) for a, b, c in zip(src, dst, w)}
    for j in rng.choice(np.arange(1, n), 290, replace=False):
        keys.setdefault((0, int(j)), float(rng.uniform(0.05, 0.3)))
    e = sorted(keys)
    src = np.array([a for a, _ in e], np.int32)
    dst = np.array([b for _, b in e], np.int32)
    w = np.array([keys[k] for k in e])
    assert np.bincount(np.r_[src, dst], minlength=n).max() > 256
    _compare_path(A, src, dst, w, [0.05, 0.5], q, "ssnal", 1e-7, tol_oracle=1e-9, x_tol=1e-5)
