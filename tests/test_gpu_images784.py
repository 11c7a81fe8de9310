"""The n = 1e5, d = 784 image workload (the benchmark's largest configuration)
solved along its 15-gamma path for q = 1, 2 and inf, certified by the oracle
(GPU).

The graph is the library's exact integer k-NN graph of the 8-bit codes (the
same launch the benchmark times); the path is solved gamma by gamma with
warm starts (X, U) to relative KKT 1e-6, as the benchmark's path does.  At
gamma indices 0, 7 and 14 the oracle, on the host, in FP64:

* recomputes the KKT residuals of the GPU's (X, U) (must be <= 1e-6);
* bounds the distance to the unique solution X* by the duality gap,
  ||X - X*||^2 <= 2 (f_p(X) - f_d(Pi_C U)) (1-strong convexity and weak
  duality), which must be <= 1e-5 ||X||; where the gap of the 1e-6 solution
  is too loose for that, the library solves the same gamma again to KKT
  1e-10 from it, the oracle bounds that solution the same way, and the
  bound for X is ||X - X_tight|| plus the tight solution's bound;
* applies its cluster rule to the GPU's X; the labels must be equal unless
  an edge sits within rounding of the fusion threshold.

A full oracle solve at this size takes hours per gamma; the certificate is
what the oracle can compute here, and it bounds the error against X*
itself rather than against another iterate."""
import numpy as np
import pytest

import oracle
import synthdata
from oracle import operators as ops
from gpu_util import need_gpu, dev, host

pytestmark = pytest.mark.gpu

GAMMAS = np.logspace(-3, 1, 15)
CHECK = (0, 7, 14)


@pytest.fixture(scope="module")
def images():
    torch, ccm = need_gpu()
    A, _, K = synthdata.images784()
    Ad = dev(A)
    src, dst, w, phi = ccm.ccm_build_knn_graph_u8(dev(K), 1.0 / 255.0, 10, 0.0)
    hs, hd, hw = host(src), host(dst), host(w)
    data = dict(A=A, Ad=Ad, src=src, dst=dst, w=w, hs=hs, hd=hd, hw=hw,
                B=oracle.incidence(hs, hd, A.shape[0]), S=oracle.fusion_scale(A))
    yield data
    del data
    torch.cuda.empty_cache()
    ccm.ccm_release_workspace()


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("q", [2.0, 1.0, np.inf])
def test_images784_path_certified(images, q):
    torch, ccm = need_gpu()
    A, Ad, B, S = images["A"], images["Ad"], images["B"], images["S"]
    src, dst, w = images["src"], images["dst"], images["w"]
    hs, hd, hw = images["hs"], images["hd"], images["hw"]
    n = A.shape[0]
    X = U = None
    report = []
    for t, g in enumerate(GAMMAS):
        out = ccm.ccm_solve_path(Ad, src, dst, w, [g], q, 1e-6, want_U=True, X_warm=X,
                                 U_warm=U)
        assert int(out["status"][0]) == 0, (q, t, out["kkt"][0])
        X, U = out["X"][0], out["U"][0]
        if t not in CHECK:
            continue
        print(f"q={q} gamma index {t}: certifying", flush=True)
        Xh, Uh = host(X), host(U)
        bound, res = ops.distance_bound(Xh, Uh, A, B, g * hw, q)
        assert res["kkt"] <= 1e-6 * 1.0001, (q, t, res)
        nX = float(np.linalg.norm(Xh))
        how = "gap"
        if bound > 1e-5 * nX:
            tight = ccm.ccm_solve_path(Ad, src, dst, w, [g], q, 1e-10, want_U=True, X_warm=X,
                                       U_warm=U)
            assert int(tight["status"][0]) == 0, (q, t)
            Xt, Ut = host(tight["X"][0]), host(tight["U"][0])
            del tight
            bt, rt = ops.distance_bound(Xt, Ut, A, B, g * hw, q)
            assert rt["kkt"] <= 1e-10 * 1.0001, (q, t, rt)
            bound = float(np.linalg.norm(Xh - Xt)) + bt
            how = "tight solve + gap"
            del Xt, Ut
        report.append((t, bound / nX, how))
        assert bound <= 1e-5 * nX, (q, t, bound / nX)
        # labels: the oracle's cluster rule on the GPU's X
        nd = np.linalg.norm(Xh[hs] - Xh[hd], axis=1)
        thr = oracle.labels.FUSE_TOL * (1.0 + S)
        if np.min(np.abs(nd - thr)) > 1e-9 * thr:
            lab, nc = oracle.cluster_labels(Xh, hs, hd, n, S)
            assert np.array_equal(host(out["labels"][0]), lab), (q, t)
            assert int(out["n_clusters"][0]) == nc
        del Xh, Uh
    print(f"q={q}: relative X error bounds {report}", flush=True)
