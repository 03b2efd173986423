"""Helpers for the GPU tests: device copies in the layouts the C ABI uses,
and the element-wise tolerance of FP64 dot products."""
import numpy as np
import pytest

EPS = 2.0 ** -53


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev_colmajor(H):
    """Device copy of H whose memory is column-major (strides (1, N))."""
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(H.T)).cuda().t()


def dev_block(V):
    """Row-major device copy of an N x n block."""
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(V, dtype=np.complex128)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def dot_bound(absA, absB, K):
    """Element-wise bound on the rounding error of complex dot products of
    length K accumulated in FP64 (each complex product-add costs at most a
    few roundings): 4 (K + 2) u (|A| |B|)."""
    return 4.0 * (K + 2) * EPS * (absA @ absB)
