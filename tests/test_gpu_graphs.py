"""CG iterations replayed from captured HIP graphs against plain launches
(GPU): the same kernels with the same arguments, so every result must be
bit-identical, over paths that replay each graph many times between the
solver's own eager launches and host reads."""
import numpy as np
import pytest

import oracle
import synthdata
from gpu_util import need_gpu, dev, host, graph_dev

pytestmark = pytest.mark.gpu


def _same(a, b):
    import torch
    assert torch.equal(a["X"], b["X"])
    if a.get("U") is not None:
        assert torch.equal(a["U"], b["U"])
    assert torch.equal(a["labels"], b["labels"])
    assert np.array_equal(a["kkt"], b["kkt"])
    assert np.array_equal(a["status"], b["status"])
    for sa, sb in zip(a["stats"], b["stats"]):
        for k in ("outer", "newton", "cg", "linesearch"):
            assert sa[k] == sb[k], k


@pytest.mark.parametrize("q,method", [(2.0, 0), (1.0, 0), (np.inf, 0), (2.0, 1), (2.0, 3)])
def test_graph_replay_matches_plain_launches(q, method):
    torch, ccm = need_gpu()
    A, _ = synthdata.mixture64(n_per=60, d=12, n_blobs=4, seed=1501)
    src, dst, w, *_ = oracle.knn_graph(A, 6, None)
    gammas = synthdata.gamma_grid(-2, 1, 5)
    Ad, gd = dev(A), graph_dev(src, dst, w)
    runs = []
    for graphs in (1, 0, 1):
        o = ccm.ccm_default_options(method=method, graphs=graphs)
        runs.append(ccm.ccm_solve_path(Ad, *gd, gammas, q, 1e-8, opts=o, want_U=True))
    _same(runs[0], runs[1])
    _same(runs[0], runs[2])
    assert all(int(s) == 0 for s in runs[0]["status"])
    assert sum(st["cg"] for st in runs[0]["stats"]) > 20  # many replays


def test_batched_groups_accept_the_graph_option():
    # the batched form runs plain launches whatever the option says (its
    # groups capture-free, see ccm_options.graphs): results bit-identical
    torch, ccm = need_gpu()
    insts = synthdata.instances(seed=1502, count=8, n_lo=40, n_hi=120, dims=(2, 8),
                                blobs_lo=2, blobs_hi=4)
    devs = []
    for it in insts:
        src, dst, w, *_ = oracle.knn_graph(it["A"], 5, None)
        devs.append(dict(A=dev(it["A"]), src=dev(src.astype(np.int32)),
                         dst=dev(dst.astype(np.int32)), w=dev(w), q=it["q"]))
    g = synthdata.gamma_grid(-2, 0.5, 3)
    a = ccm.ccm_solve_path_batched(devs, g, 1e-7, opts=ccm.ccm_default_options(graphs=1))
    b = ccm.ccm_solve_path_batched(devs, g, 1e-7, opts=ccm.ccm_default_options(graphs=0))
    for ra, rb in zip(a, b):
        assert torch.equal(ra["X"], rb["X"])
        assert torch.equal(ra["labels"], rb["labels"])
        assert np.array_equal(ra["kkt"], rb["kkt"])
        assert np.all(ra["status"] == 0)
