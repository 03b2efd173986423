"""Helpers for the GPU tests: device copies in the layouts the C ABI uses,
and the element-wise tolerance of FP64 dot products."""
import hashlib

import numpy as np
import pytest

from oracle import eig

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


_ORACLE_CACHE = {}


def _key(H, what, m=0):
    return (what, H.shape, m, hashlib.blake2b(np.ascontiguousarray(H).tobytes(),
                                              digest_size=16).hexdigest())


def _oracle_lowest(H, m):
    k = _key(H, "lowest", m)
    if k not in _ORACLE_CACHE:
        _ORACLE_CACHE[k] = eig.eigh_lowest(H, m)
    return _ORACLE_CACHE[k]


def _oracle_norm(H):
    """||H||_2 = max |lambda| (LAPACK eigenvalues, a library routine)."""
    k = _key(H, "norm")
    if k not in _ORACLE_CACHE:
        _ORACLE_CACHE[k] = float(np.abs(np.linalg.eigvalsh(H)).max())
    return _ORACLE_CACHE[k]


def check_against_oracle(H, res, nev, hn=None):
    """End-to-end bar against the oracle (per eigenpair): relative eigenvalue
    error <= 1e-10, ||H v - lambda v|| / ||H||_2 <= 1e-10, max |V^H V - I|
    <= 1e-12, each cluster's subspace within the Davis-Kahan bound of the
    oracle's, and the phase convention.  ``res`` has ``eigvals`` and a
    device ``V``; the oracle's eigenpairs are cached per matrix."""
    w, V = res.eigvals, host(res.V)
    N = H.shape[0]
    m = min(nev + 1, N)
    w_ext, V_ext = _oracle_lowest(H, m)
    w_ref, V_ref = w_ext[:nev], V_ext[:, :nev]
    if hn is None:
        hn = _oracle_norm(H)
    assert np.all(np.abs(w - w_ref) <= 1e-10 * np.abs(w_ref) + 1e-300), np.abs(w - w_ref).max()
    R = H @ V - V * w[None, :]
    rn = np.linalg.norm(R, axis=0)
    assert rn.max() / hn <= 1e-10
    assert np.abs(V.conj().T @ V - np.eye(nev)).max() <= 1e-12
    # Eigenvectors: group eigenvalues closer than 1e-6 ||H|| into clusters
    # and compare each cluster's subspace with the oracle's; by Davis-Kahan
    # each side's angle to the exact subspace is at most its residual norm
    # over the gap to the rest of the spectrum (a single vector is unique up
    # to phase).  Computed residuals carry ~sqrt(N) u ||H|| of rounding.
    rn_ref = np.linalg.norm(H @ V_ref - V_ref * w_ref[None, :], axis=0)
    floor = 2.0 * np.sqrt(N) * 2.0 ** -53 * hn
    start = 0
    while start < nev:
        end = start + 1
        while end < nev and w_ref[end] - w_ref[end - 1] <= 1e-6 * hn:
            end += 1
        gap = np.inf
        if start > 0:
            gap = min(gap, w_ref[start] - w_ref[start - 1])
        if end < m:
            gap = min(gap, w_ext[end] - w_ext[end - 1])
        A, B = V[:, start:end], V_ref[:, start:end]
        d = np.linalg.norm(A @ (A.conj().T @ B) - B, 2)
        k = end - start
        r_both = (np.linalg.norm(rn[start:end]) + np.linalg.norm(rn_ref[start:end])
                  + 2.0 * np.sqrt(k) * floor)
        bound = 2.0 * r_both / max(gap, 1e-300) + 1e-13
        assert d <= bound, (start, end, d, bound)
        start = end
    # Phase convention: the entry of largest modulus is real and positive.
    for j in range(nev):
        i = np.argmax(np.abs(V[:, j]))
        assert V[i, j].imag == 0.0 and V[i, j].real > 0.0
