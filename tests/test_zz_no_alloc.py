"""ccm_labels_noalloc (fixed work space, no allocation in the call) against
ccm_labels and the oracle (GPU), called through the C ABI."""
import numpy as np
import pytest

import oracle
import synthdata
from gpu_util import need_gpu, dev, host

pytestmark = pytest.mark.gpu


def _case(n_per, d, blobs, seed):
    """Points, a solution-like X (most blobs collapsed to their mean, every
    seventh point left where it is) and a k-NN edge list."""
    A, y = synthdata.mixture64(n_per=n_per, d=d, n_blobs=blobs, seed=seed)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    X = A.copy()
    for b in range(blobs - 1):
        X[y == b] = A[y == b].mean(0)
    X[::7] = A[::7]
    return A, X, src, dst


def test_noalloc_labels_match_allocating_entry_point_twice():
    torch, ccm = need_gpu()
    # the second call is smaller: the array keeps the first call's contents
    for n_per, d, blobs, seed in [(400, 16, 6, 3001), (40, 5, 4, 3002)]:
        A, X, src, dst = _case(n_per, d, blobs, seed)
        n = A.shape[0]
        dA, dX = dev(A), dev(X)
        s, t = dev(src.astype(np.int32)), dev(dst.astype(np.int32))
        ref, nref = ccm.ccm_labels(dA, dX, s, t)
        lab, nc = ccm.ccm_labels_noalloc(dA, dX, s, t)
        assert nc == nref, (n, nc, nref)
        assert torch.equal(lab, ref)
        olab, on = oracle.cluster_labels(X, src, dst, n, oracle.fusion_scale(A))
        assert nc == on and np.array_equal(host(lab), olab)
        assert 1 < nc < n


def test_noalloc_labels_without_edges_and_over_capacity():
    torch, ccm = need_gpu()
    from paper_2501_15964_amd.ccm import CcmError
    A = np.random.default_rng(3003).normal(size=(9, 3))
    e = dev(np.zeros(0, np.int32))
    lab, nc = ccm.ccm_labels_noalloc(dev(A), dev(A), e, e)
    assert nc == 9 and np.array_equal(host(lab), np.arange(9))
    big = torch.zeros(((1 << 22) + 1, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(CcmError) as ex:
        ccm.ccm_labels_noalloc(big, big, e, e)
    assert ex.value.status == 5  # CCM_E_CAPACITY
