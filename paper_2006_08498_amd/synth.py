"""Seeded synthetic inputs: BSE-shaped Hermitian matrices and random blocks.

This module builds inputs only.  It holds none of the eigensolver's
arithmetic, so both the HIP path and the CPU oracle may take their inputs
from here.

Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), a counter-based
generator: every matrix entry is a pure function of (seed, stream, i, j), so
a matrix can be produced panel by panel, on the host or on the device, and
comes out the same whatever the thread count.  Normals come from the
Box-Muller transform applied to two 53-bit uniforms.

Matrix families (stand-ins for the paper's BSE Hamiltonians, whose spectra
have a small wanted band at the bottom and a largest eigenvalue several
times the last wanted one; see the supplement's convergence tables):

* ``dk``: H = D + K, D = diag of "transition energies" uniform in [1, 6),
  K Hermitian with complex Gaussian entries of standard deviation
  ``std * exp(-|i-j| / decay)``.  The diagonal of K is real Gaussian.
* ``planted``: H = Q diag(lam) Q^H with Q Haar-distributed (QR of a complex
  Gaussian matrix with the phases of diag(R) divided out, Mezzadri 2007)
  and lam: ``n_clusters`` clusters of ``cluster_size`` values 1e-4 apart
  starting at 2.0 with spacing 0.025, the rest uniform in [2.5, 8.0).

Layout convention: functions return numpy arrays indexed ``H[i, j]`` =
row i, column j.  ``colmajor(H)`` gives the byte layout the C ABI expects.
"""
from __future__ import annotations

import numpy as np

# Philox4x32 round multipliers and Weyl key increments (SC'11, Sec. 5).
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

# Stream tags: the third counter word separates independent draws.
STREAM_DIAG = 0        # D of D + K
STREAM_K = 1           # K of D + K
STREAM_LAMBDA = 2      # planted spectrum, uniform part
STREAM_GAUSS = 3       # planted spectrum, Gaussian matrix for Q
STREAM_BLOCK = 4       # random N x n blocks (start vectors for tests)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds, vectorised over numpy arrays.

    Counters and keys are 32-bit values (any integer dtype that holds them).
    Returns four uint64 arrays holding 32-bit outputs.
    """
    x0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    x0, x1, x2, x3 = (x0.copy(), x1.copy(), x2.copy(), x3.copy())
    key0 = int(k0) & 0xFFFFFFFF
    key1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            key0 = (key0 + _PHILOX_W0) & 0xFFFFFFFF
            key1 = (key1 + _PHILOX_W1) & 0xFFFFFFFF
        p0 = _PHILOX_M0 * x0          # < 2^64, exact in uint64
        p1 = _PHILOX_M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(key0), lo1,
                          hi0 ^ x3 ^ np.uint64(key1), lo0)
    return x0, x1, x2, x3


def _u53(a, b):
    """Uniform in the open interval (0, 1) from two 32-bit words."""
    hi = (a >> np.uint64(5)).astype(np.float64)   # 27 bits
    lo = (b >> np.uint64(6)).astype(np.float64)   # 26 bits
    return (hi * 67108864.0 + lo + 0.5) / 9007199254740992.0


def _keys(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def uniform_pair(i, j, stream, seed):
    """Two independent U(0,1) doubles for counter (i, j, stream)."""
    k0, k1 = _keys(seed)
    w = philox4x32_10(i, j, stream, 0, k0, k1)
    return _u53(w[0], w[1]), _u53(w[2], w[3])


def normal_pair(i, j, stream, seed):
    """Two independent N(0,1) doubles for counter (i, j, stream)."""
    u1, u2 = uniform_pair(i, j, stream, seed)
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def complex_normal(i, j, stream, seed):
    """Complex Gaussian with E|z|^2 = 1 for counter (i, j, stream)."""
    z0, z1 = normal_pair(i, j, stream, seed)
    return (z0 + 1j * z1) * np.sqrt(0.5)


# --------------------------------------------------------------------------
# D + K family
# --------------------------------------------------------------------------

def dk_diag(N, seed, lo=1.0, hi=6.0):
    """Transition energies d_i, uniform in [lo, hi), unsorted."""
    i = np.arange(N, dtype=np.uint64)
    u, _ = uniform_pair(i, 0, STREAM_DIAG, seed)
    return lo + (hi - lo) * u


def dk_entries(i, j, seed, std, decay):
    """Entries H[i, j] of D + K for index arrays with i >= j (lower part)."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    z0, z1 = normal_pair(i.astype(np.uint64), j.astype(np.uint64), STREAM_K, seed)
    s = std * np.exp(-np.abs(i - j).astype(np.float64) / decay)
    off = s * (z0 + 1j * z1) * np.sqrt(0.5)
    diag = std * z0 + 0j
    return np.where(i == j, diag, off)


def dk_rows(rows, N, seed=0, std=0.02, decay=200.0):
    """Selected full rows H[rows, :] of D + K (same entries as dk_matrix),
    without forming the matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    d = dk_diag(N, seed)
    out = np.empty((rows.size, N), dtype=np.complex128)
    j = np.arange(N, dtype=np.int64)
    for t, i in enumerate(rows):
        lo = j <= i
        ii = np.full(N, i, dtype=np.int64)
        # lower part (j <= i) is generated at (i, j); upper part is the
        # conjugate of the entry generated at (j, i)
        low = dk_entries(ii[lo], j[lo], seed, std, decay)
        up = np.conj(dk_entries(j[~lo], ii[~lo], seed, std, decay))
        out[t, lo] = low
        out[t, ~lo] = up
        out[t, i] = np.real(low[i]) + d[i]
    return out


def dk_matrix(N, seed=0, std=0.02, decay=200.0, row_block=512):
    """Dense D + K (complex128, Hermitian to the last bit)."""
    H = np.zeros((N, N), dtype=np.complex128)
    d = dk_diag(N, seed)
    for r0 in range(0, N, row_block):
        r1 = min(N, r0 + row_block)
        ii, jj = np.meshgrid(np.arange(r0, r1), np.arange(N), indexing="ij")
        mask = jj <= ii
        vals = dk_entries(ii[mask], jj[mask], seed, std, decay)
        blk = np.zeros((r1 - r0, N), dtype=np.complex128)
        blk[mask] = vals
        H[r0:r1, :] = blk
    # Mirror the strict lower triangle into the upper one.
    low = np.tril(H, -1)
    H = low + low.conj().T + np.diag(np.real(np.diag(H)) + d)
    return H


# --------------------------------------------------------------------------
# Planted-spectrum family
# --------------------------------------------------------------------------

def planted_spectrum(N, seed=0, n_clusters=20, cluster_size=10, start=2.0,
                     spacing=0.025, gap=1e-4, rest_lo=2.5, rest_hi=8.0):
    """Eigenvalues of the planted family, ascending."""
    k = np.arange(n_clusters)[:, None]
    j = np.arange(cluster_size)[None, :]
    low = (start + spacing * k + gap * j).ravel()
    nlow = min(N, low.size)
    low = low[:nlow]
    nrest = N - nlow
    i = np.arange(nrest, dtype=np.uint64)
    u, _ = uniform_pair(i, 0, STREAM_LAMBDA, seed)
    rest = rest_lo + (rest_hi - rest_lo) * u
    return np.sort(np.concatenate([low, rest]))


def gaussian_matrix(N, M, seed, stream=STREAM_GAUSS):
    """N x M complex Gaussian matrix, entry (i, j) from counter (i, j, stream)."""
    ii, jj = np.meshgrid(np.arange(N, dtype=np.uint64),
                         np.arange(M, dtype=np.uint64), indexing="ij")
    return complex_normal(ii, jj, stream, seed)


def haar_unitary(N, seed=0):
    """Haar unitary: QR of a complex Gaussian, phases of diag(R) removed."""
    G = gaussian_matrix(N, N, seed)
    Q, R = np.linalg.qr(G)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def planted_matrix(N, seed=0, lam=None, **spec):
    """H = Q diag(lam) Q^H, symmetrised; returns (H, lam ascending, Q)."""
    if lam is None:
        lam = planted_spectrum(N, seed, **spec)
    Q = haar_unitary(N, seed)
    H = (Q * lam[None, :]) @ Q.conj().T
    H = 0.5 * (H + H.conj().T)
    return H, np.asarray(lam, dtype=np.float64), Q


# --------------------------------------------------------------------------
# Structured special cases
# --------------------------------------------------------------------------

def hermitian_circulant_row(N, seed=0):
    """First row c of a Hermitian circulant: c_0 real, c_{N-k} = conj(c_k)."""
    c = complex_normal(np.arange(N, dtype=np.uint64), 0, STREAM_BLOCK, seed)
    c[0] = c[0].real + 3.0
    for k in range(1, N):
        if k < N - k:
            c[N - k] = np.conj(c[k])
        elif k == N - k:
            c[k] = c[k].real
    return c


def circulant(c):
    """C[i, j] = c[(j - i) mod N]."""
    N = len(c)
    idx = (np.arange(N)[None, :] - np.arange(N)[:, None]) % N
    return np.asarray(c)[idx]


def tridiag_toeplitz(N, a, b):
    """a on the diagonal, b below it, conj(b) above it."""
    H = np.diag(np.full(N, a, dtype=np.complex128))
    H += np.diag(np.full(N - 1, b, dtype=np.complex128), -1)
    H += np.diag(np.full(N - 1, np.conj(b), dtype=np.complex128), 1)
    return H


def random_block(N, n, seed=0, stream=STREAM_BLOCK):
    """N x n complex Gaussian block (start vectors for tests)."""
    return gaussian_matrix(N, n, seed, stream)


def gaussian_integer_hermitian(N, seed=0, lim=4):
    """Hermitian matrix with small Gaussian-integer entries (exact tests)."""
    ii, jj = np.meshgrid(np.arange(N, dtype=np.uint64),
                         np.arange(N, dtype=np.uint64), indexing="ij")
    u1, u2 = uniform_pair(ii, jj, STREAM_BLOCK, seed)
    re = np.floor(u1 * (2 * lim + 1)) - lim
    im = np.floor(u2 * (2 * lim + 1)) - lim
    A = re + 1j * im
    low = np.tril(A, -1)
    return low + low.conj().T + np.diag(np.real(np.diag(A)))


def colmajor(A):
    """Fortran-ordered copy: the byte layout of a column-major matrix."""
    return np.asfortranarray(A, dtype=np.complex128)


# --------------------------------------------------------------------------
# Device generators (large N): same definitions, evaluated by the HIP
# kernels of libchase_synth.so.  torch supplies memory and the stream; the
# planted family also uses torch's dense QR and matrix product on the device,
# which build the input and are not part of the solver.
# --------------------------------------------------------------------------

_synth_lib = None


def _slib():
    global _synth_lib
    if _synth_lib is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchase_synth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run paper_2006_08498_amd/build.py")
        L = ctypes.CDLL(path)
        P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.synth_dk.restype = ctypes.c_int
        L.synth_dk.argtypes = [P, I64, I64, ctypes.c_uint64, D, D, D, D, P]
        L.synth_gauss.restype = ctypes.c_int
        L.synth_gauss.argtypes = [P, I64, I64, I64, ctypes.c_uint64, ctypes.c_uint32, P]
        L.synth_copy.restype = ctypes.c_int
        L.synth_copy.argtypes = [P, P, I64, P]
        _synth_lib = L
    return _synth_lib


def _stream():
    import ctypes
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def dk_matrix_device(N, seed=0, std=0.02, decay=200.0, device="cuda"):
    """D + K on the device, returned column-major (strides (1, N))."""
    import ctypes
    import torch
    H = torch.empty((N, N), dtype=torch.complex128, device=device).t()
    st = _slib().synth_dk(ctypes.c_void_p(H.data_ptr()), N, N, int(seed), std,
                          decay, 1.0, 6.0, _stream())
    if st != 0:
        raise RuntimeError(f"synth_dk failed ({st})")
    return H


def gaussian_matrix_device(N, M, seed, stream=STREAM_GAUSS, device="cuda"):
    """N x M complex Gaussian on the device, column-major (strides (1, N))."""
    import ctypes
    import torch
    G = torch.empty((M, N), dtype=torch.complex128, device=device).t()
    st = _slib().synth_gauss(ctypes.c_void_p(G.data_ptr()), N, N, M, int(seed),
                             int(stream), _stream())
    if st != 0:
        raise RuntimeError(f"synth_gauss failed ({st})")
    return G


def planted_matrix_device(N, seed=0, lam=None, device="cuda", **spec):
    """Planted-spectrum H on the device (row-major torch tensor) and its
    eigenvalues; Q from the device QR of a Philox Gaussian matrix."""
    import torch
    if lam is None:
        lam = planted_spectrum(N, seed, **spec)
    G = gaussian_matrix_device(N, N, seed, device=device)
    Q, R = torch.linalg.qr(G)
    del G
    d = torch.diagonal(R)
    Q *= (d / d.abs())[None, :]
    del R
    lt = torch.as_tensor(np.asarray(lam), dtype=torch.float64, device=device)
    H = (Q * lt[None, :]) @ Q.conj().t()
    del Q
    H = 0.5 * (H + H.conj().t())
    return H.contiguous(), np.asarray(lam, dtype=np.float64)


def device_copy(src, dst):
    """Plain device copy kernel (traffic calibration for HBM counters)."""
    import ctypes
    n = src.numel() * src.element_size()
    st = _slib().synth_copy(ctypes.c_void_p(src.data_ptr()),
                            ctypes.c_void_p(dst.data_ptr()), n, _stream())
    if st != 0:
        raise RuntimeError(f"synth_copy failed ({st})")
