"""Helpers shared by the GPU tests: device transfer and the library handle.

The GPU tests exercise libccm through its C ABI (via the ctypes binding) and
compare with the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2501_15964_amd as ccm
    ccm.lib()  # raises if the library is missing: no fallback exists
    return torch, ccm


def dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def graph_dev(src, dst, w):
    import torch
    return (dev(np.asarray(src, dtype=np.int32)), dev(np.asarray(dst, dtype=np.int32)),
            dev(np.asarray(w, dtype=np.float64)))


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
