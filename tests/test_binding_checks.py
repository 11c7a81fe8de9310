"""Argument checks of the Python binding that run before any device call
(CPU): wrong dtypes or shapes raise ValueError instead of reaching the
library with buffers of another layout."""
import numpy as np
import pytest
import torch

import paper_2501_15964_amd as ccm


def _graph(n=6, m=5):
    A = torch.zeros((n, 2), dtype=torch.float64)
    src = torch.arange(m, dtype=torch.int32)
    dst = src + 1
    w = torch.ones(m, dtype=torch.float64)
    return A, src, dst, w


@pytest.mark.parametrize("bad", ["src64", "dst64", "w32", "A32", "A1d", "short_w"])
def test_solve_path_rejects_wrong_dtypes_and_shapes(bad):
    A, src, dst, w = _graph()
    if bad == "src64":
        src = src.long()
    elif bad == "dst64":
        dst = dst.long()
    elif bad == "w32":
        w = w.float()
    elif bad == "A32":
        A = A.float()
    elif bad == "A1d":
        A = A.reshape(-1)
    elif bad == "short_w":
        w = w[:-1]
    with pytest.raises(ValueError):
        ccm.ccm_solve_path(A, src, dst, w, [0.1], 2.0, 1e-6)


def test_solve_path_rejects_bad_warm_start():
    A, src, dst, w = _graph()
    with pytest.raises(ValueError):
        ccm.ccm_solve_path(A, src, dst, w, [0.1], 2.0, 1e-6, X_warm=A.float())
    with pytest.raises(ValueError):
        ccm.ccm_solve_path(A, src, dst, w, [0.1], 2.0, 1e-6, X_warm=A[:-1])
    with pytest.raises(ValueError):
        ccm.ccm_solve_path(A, src, dst, w, [0.1], 2.0, 1e-6,
                           U_warm=torch.zeros((5, 3), dtype=torch.float64))


def test_batched_rejects_wrong_dtypes():
    A, src, dst, w = _graph()
    good = dict(A=A, src=src, dst=dst, w=w, q=2.0)
    for key, val in [("src", src.long()), ("w", w.float()), ("A", A.float())]:
        bad = dict(good)
        bad[key] = val
        with pytest.raises(ValueError):
            ccm.ccm_solve_path_batched([good, bad], [0.1], 1e-6)


def test_weights_from_log_needs_float64():
    with pytest.raises(ValueError):
        ccm.ccm_weights_from_log(torch.zeros(3, dtype=torch.float32))


def test_status_codes_named():
    L = ccm.lib()
    assert L.ccm_status_string(ccm.CCM_E_NOT_CONVERGED).decode() != "unknown status"
    assert ccm.CCM_E_NOT_CONVERGED == 6


def test_status_codes_match_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "ccm.h")).read()
    for name, val in re.findall(r"\b(CCM_(?:OK|E_[A-Z_]+))\s*=\s*(\d+)", hdr):
        assert getattr(ccm, name) == int(val), name
