"""Python binding of libchase_mi355x (argument marshalling only).

Every step of the solver runs in the library's HIP kernels; torch provides
device memory and the stream.  The binding fails loudly when the library
is missing: there is no CPU fallback.

Layout of H: the C ABI reads H column-major.  A torch tensor with strides
(1, N) is passed as is.  A row-major tensor (strides (N, 1)) read
column-major is H^T = conj(H) for a Hermitian H: the eigenvalues are the
same and the eigenvectors are conjugated, which the binding undoes.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchase_mi355x.so")

CHASE_PENDING = -1
CHASE_OK = 0
CHASE_EINVAL = 1
CHASE_ENOMEM = 2
CHASE_EHIP = 3
CHASE_ENOCONV = 4
CHASE_ENONFINITE = 5
CHASE_EBOUNDS = 6
CHASE_EINTERNAL = 7
CHASE_FP64 = 0
CHASE_MIXED = 1
CHASE_SERVER_FUSE_FILTER = 1
CHASE_SERVER_SHORTEST_FIRST = 2

STATUS_NAMES = {
    CHASE_PENDING: "CHASE_PENDING", CHASE_OK: "CHASE_OK",
    CHASE_EINVAL: "CHASE_EINVAL", CHASE_ENOMEM: "CHASE_ENOMEM",
    CHASE_EHIP: "CHASE_EHIP", CHASE_ENOCONV: "CHASE_ENOCONV",
    CHASE_ENONFINITE: "CHASE_ENONFINITE", CHASE_EBOUNDS: "CHASE_EBOUNDS",
    CHASE_EINTERNAL: "CHASE_EINTERNAL",
}


class ChaseOpts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("initial_degree", ctypes.c_int32),
        ("degree_extra", ctypes.c_int32),
        ("lanczos_steps", ctypes.c_int32),
        ("lanczos_runs", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("switch_tol", ctypes.c_double),
        ("dV0", ctypes.c_void_p),
        ("profile", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
        ("on_iteration", ctypes.c_void_p),
        ("on_iteration_user", ctypes.c_void_p),
        ("v0_cols", ctypes.c_int32),
        ("out_cols", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class ChaseInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32),
        ("nconv", ctypes.c_int32),
        ("matvecs_filter", ctypes.c_int64),
        ("matvecs_filter_fp32", ctypes.c_int64),
        ("matvecs_total", ctypes.c_int64),
        ("filter_launches", ctypes.c_int64),
        ("mu1", ctypes.c_double),
        ("mu_ne", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("hnorm_est", ctypes.c_double),
        ("t_lanczos", ctypes.c_double),
        ("t_filter", ctypes.c_double),
        ("t_qr", ctypes.c_double),
        ("t_rr", ctypes.c_double),
        ("t_resid", ctypes.c_double),
        ("t_total", ctypes.c_double),
        ("t_filter_kernels", ctypes.c_double),
        ("filter_flops", ctypes.c_double),
        ("t_shadow", ctypes.c_double),
        ("t_filter32_kernels", ctypes.c_double),
        ("filter32_launches", ctypes.c_int64),
        ("gemm_time", ctypes.c_double),
        ("gemm_flops", ctypes.c_double),
        ("gemm_launches", ctypes.c_int64),
        ("refinements", ctypes.c_int64),
        ("lanczos_flops", ctypes.c_double),
        ("lanczos_bytes", ctypes.c_double),
        ("filter_bytes", ctypes.c_double),
        ("qr_flops", ctypes.c_double),
        ("qr_bytes", ctypes.c_double),
        ("rr_flops", ctypes.c_double),
        ("rr_bytes", ctypes.c_double),
        ("resid_flops", ctypes.c_double),
        ("resid_bytes", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ChaseError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

# Exported symbols and their signatures (must match include/chase_mi355x.h).
SIGNATURES = {
    "chase_default_opts": (None, [ctypes.POINTER(ChaseOpts)]),
    "chase_last_error": (ctypes.c_char_p, []),
    "chase_solve": (ctypes.c_int, [_P, _I64, _I32, _I32, _D, _I32, _P, _P]),
    "chase_workspace_bytes": (ctypes.c_size_t, [_I64, _I32, _I32, ctypes.POINTER(ChaseOpts)]),
    "chase_solve_ex": (ctypes.c_int, [_P, _I64, _I64, _I32, _I32, _D, _I32, _P, _P,
                                      _P, _I64, _P, ctypes.c_size_t, _P,
                                      ctypes.POINTER(ChaseOpts), ctypes.POINTER(ChaseInfo)]),
    "chase_filter_step": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, _I64,
                                         _I32, _D, _D, _D, _P]),
    "chase_filter_step_group": (ctypes.c_int, [_P, _I32, _P]),
    "chase_filter_step_c": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, _I64,
                                           _I32, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, _P]),
    "chase_shadow_c": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _P]),
    "chase_filter": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I32, _P, _D, _D, _D,
                                    ctypes.POINTER(ctypes.c_int64), _P]),
    "chase_filter_fused": (ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_int64), _P]),
    "chase_lanczos": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I32, _I32, _P, _P, _P]),
    "chase_lanczos_bounds": (ctypes.c_int, [_P, _P, _I32, _I32, _I64, _I32, _P]),
    "chase_qr": (ctypes.c_int, [_P, _I64, _I64, _I32, _I32, _P]),
    "chase_rayleigh_ritz": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I32, _P, _P, _P]),
    "chase_residuals": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I32, _P, _P, _P]),
    "chase_heevj": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "chase_heevj_noalloc": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "chase_degrees": (ctypes.c_int, [_P, _P, _I32, _D, _D, _D, _I32, _I32, _P]),
    "chase_nex_linear": (_I32, [_I32, _I32, _D, _D, _D]),
    "chase_ingest_rows": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I64, _I64, _P]),
    "chase_ingest_rows_host": (ctypes.c_int, [_P, _I64, _I64, _P, _I64, _I64, _I64, _P]),
    "chase_hermitian_complete": (ctypes.c_int, [_P, _I64, _I64, _I32, _P]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with "
            "`python paper_2006_08498_amd/build.py` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    msg = lib().chase_last_error()
    return msg.decode() if msg else ""


def _check(st, allow=(CHASE_OK,)):
    if st not in allow:
        raise ChaseError(st, last_error())
    return st


def default_opts(**kw) -> ChaseOpts:
    o = ChaseOpts()
    lib().chase_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ torch

def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _h_layout(H):
    """(pointer, ldh, conjugated?) for a square complex128 CUDA tensor."""
    torch = _torch()
    if H.dtype != torch.complex128 or not H.is_cuda or H.dim() != 2:
        raise ValueError("H must be a 2-D complex128 CUDA tensor")
    N = H.shape[0]
    if H.shape[1] != N:
        raise ValueError("H must be square")
    s0, s1 = H.stride()
    if s0 == 1 and s1 >= N:
        return _dptr(H), s1, False
    if s1 == 1 and s0 >= N:
        return _dptr(H), s0, True
    raise ValueError("H must be column-major (strides (1, ld)) or row-major (ld, 1)")


@dataclass
class SolveResult:
    eigvals: np.ndarray
    V: object                 # torch (N, nev) complex128 on the device
    resid: np.ndarray
    status: int
    info: dict = field(default_factory=dict)


def workspace_bytes(N, nev, nex, opts=None) -> int:
    o = opts if opts is not None else default_opts()
    return int(lib().chase_workspace_bytes(N, nev, nex, ctypes.byref(o)))


ITER_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ChaseInfo))


def solve(H, nev, nex, tol=1e-10, degree_max=20, *, opts=None, V0=None,
          workspace=None, stream=None, allow_noconv=False, on_iteration=None,
          out_cols=None, **opt_kw):
    """Lowest ``nev`` eigenpairs of the Hermitian CUDA tensor ``H``.

    Returns eigenvalues (ascending), eigenvectors as an (N, nev) tensor,
    residual norms, the status and the solver's info record.
    ``on_iteration(info_dict)`` is called after every subspace iteration; a
    true return value stops the solve there (status CHASE_ENOCONV unless nev
    pairs are locked).  ``V0`` (N, k) with k <= nev + nex warm-starts the
    solve; ``out_cols`` (nev..nev+nex) returns that many columns of the final
    search block, the warm start of the next matrix of a sequence."""
    torch = _torch()
    N = H.shape[0]
    hp, ldh, conj = _h_layout(H)
    o = opts if opts is not None else default_opts(**opt_kw)
    cb_keep = None
    if on_iteration is not None:
        def _cb(_user, info_p):
            try:
                return 1 if on_iteration(info_p.contents.as_dict()) else 0
            except Exception:               # never unwind through C
                return 1
        cb_keep = ITER_FN(_cb)
        o.on_iteration = ctypes.cast(cb_keep, ctypes.c_void_p)
    v0_keep = None
    if V0 is not None:
        # Warm start, N x (nev+nex): the ABI wants it column-major (and
        # conjugated when H is passed row-major, i.e. as conj(H)).
        v0 = V0.conj() if conj else V0
        v0_keep = v0.t().contiguous()       # (k, N) row-major == col-major
        o.dV0 = v0_keep.data_ptr()
        o.v0_cols = v0_keep.shape[0]
    if out_cols is not None:
        o.out_cols = out_cols
    mout = o.out_cols if o.out_cols > 0 else nev
    out = torch.empty((mout, N), dtype=torch.complex128, device=H.device)
    ev = np.zeros(nev, dtype=np.float64)
    rs = np.zeros(nev, dtype=np.float64)
    info = ChaseInfo()
    wptr, wbytes = None, 0
    if workspace is not None:
        wptr, wbytes = _dptr(workspace), workspace.numel() * workspace.element_size()
    st = lib().chase_solve_ex(
        hp, N, ldh, nev, nex, tol, degree_max,
        ev.ctypes.data_as(_P), rs.ctypes.data_as(_P), _dptr(out), N,
        wptr, wbytes, _stream_ptr(stream), ctypes.byref(o), ctypes.byref(info))
    del cb_keep
    _check(st, (CHASE_OK, CHASE_ENOCONV) if allow_noconv else (CHASE_OK,))
    V = out.t()
    if conj:
        V = V.conj().resolve_conj()
    del v0_keep
    return SolveResult(ev, V, rs, st, info.as_dict())


# ------------------------------------------------------------ step level
# Vector blocks are row-major (N, n) contiguous torch tensors.

def _block(t, name):
    torch = _torch()
    if t.dtype != torch.complex128 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major complex128 CUDA block")
    return _dptr(t), t.stride(0)


def _h_colmajor(H):
    hp, ldh, conj = _h_layout(H)
    if conj:
        raise ValueError("step-level calls take H column-major (strides (1, ld))")
    return hp, ldh


def filter_step(H, Y, X, a, b, g, W=None, stream=None):
    """W = a H Y + b Y + g X (W defaults to a new block; may be X)."""
    torch = _torch()
    hp, ldh = _h_colmajor(H)
    N, n = Y.shape
    yp, ldy = _block(Y, "Y")
    xp, ldx = _block(X, "X") if X is not None else (None, n)
    if W is None:
        W = torch.empty_like(Y)
    wp, ldw = _block(W, "W")
    _check(lib().chase_filter_step(hp, N, ldh, yp, ldy, xp, ldx, wp, ldw, n,
                                   a, b, g, _stream_ptr(stream)))
    return W


def _block_c(t, name):
    torch = _torch()
    if t.dtype != torch.complex64 or not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major complex64 CUDA block")
    return _dptr(t), t.stride(0)


def shadow_c(H, stream=None):
    """Complex64 copy of a column-major complex128 H (column-major result)."""
    torch = _torch()
    hp, ldh = _h_colmajor(H)
    N = H.shape[0]
    Hc = torch.empty((N, N), dtype=torch.complex64, device=H.device).t()
    _check(lib().chase_shadow_c(hp, N, ldh, _dptr(Hc), N, _stream_ptr(stream)))
    return Hc


class FilterCall(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_void_p), ("N", ctypes.c_int64), ("ldh", ctypes.c_int64),
                ("dY", ctypes.c_void_p), ("ldy", ctypes.c_int64),
                ("dX", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("dW", ctypes.c_void_p), ("ldw", ctypes.c_int64), ("ncols", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("g", ctypes.c_double)]


def filter_step_group(steps, stream=None):
    """Several filter steps in grouped launches.  ``steps`` is a list of
    (H, Y, X, W, a, b, g) with the shapes of filter_step (X may be None when
    g == 0; W must be given)."""
    arr = (FilterCall * max(1, len(steps)))()
    for i, (H, Y, X, W, a, b, g) in enumerate(steps):
        hp, ldh = _h_colmajor(H)
        N, n = Y.shape
        yp, ldy = _block(Y, "Y")
        xp, ldx = _block(X, "X") if X is not None else (None, n)
        wp, ldw = _block(W, "W")
        arr[i] = FilterCall(hp, N, ldh, yp, ldy, xp, ldx, wp, ldw, n, a, b, g)
    _check(lib().chase_filter_step_group(ctypes.cast(arr, _P), len(steps),
                                         _stream_ptr(stream)))


def filter_step_c(Hc, Y, X, a, b, g, W=None, stream=None):
    """FP32 step W = a Hc Y + b Y + g X on complex64 blocks."""
    torch = _torch()
    if Hc.dtype != torch.complex64 or Hc.stride(0) != 1:
        raise ValueError("Hc must be a column-major complex64 CUDA tensor")
    N, n = Y.shape
    yp, ldy = _block_c(Y, "Y")
    xp, ldx = _block_c(X, "X") if X is not None else (None, n)
    if W is None:
        W = torch.empty_like(Y)
    wp, ldw = _block_c(W, "W")
    _check(lib().chase_filter_step_c(_dptr(Hc), N, Hc.stride(1), yp, ldy, xp, ldx, wp,
                                     ldw, n, a, b, g, _stream_ptr(stream)))
    return W


def filter(H, V, degrees, mu1, alpha, beta, stream=None):
    """Per-vector-degree Chebyshev filter of V in place; returns mat-vecs."""
    hp, ldh = _h_colmajor(H)
    N, n = V.shape
    vp, ldv = _block(V, "V")
    deg = np.ascontiguousarray(degrees, dtype=np.int32)
    mv = ctypes.c_int64(0)
    _check(lib().chase_filter(hp, N, ldh, vp, ldv, n, deg.ctypes.data_as(_P),
                              mu1, alpha, beta, ctypes.byref(mv), _stream_ptr(stream)))
    return int(mv.value)


class FilterJob(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_void_p), ("N", ctypes.c_int64), ("ldh", ctypes.c_int64),
                ("dV", ctypes.c_void_p), ("ldv", ctypes.c_int64), ("n", ctypes.c_int32),
                ("h_degrees", ctypes.c_void_p), ("mu1", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double)]


def filter_fused(jobs, stream=None):
    """Several whole filter calls in one persistent launch: ``jobs`` is a
    list of (H, V, degrees, mu1, alpha, beta) as for ``filter``; every V is
    filtered in place.  Returns the total column products."""
    arr = (FilterJob * max(1, len(jobs)))()
    keep = []
    for i, (H, V, degrees, mu1, alpha, beta) in enumerate(jobs):
        hp, ldh = _h_colmajor(H)
        if V.shape[1] == 0:                 # an empty job: nothing to read
            vp, ldv = ctypes.c_void_p(None), 0
        else:
            vp, ldv = _block(V, "V")
        d = np.ascontiguousarray(degrees, dtype=np.int32)
        keep.append(d)
        arr[i] = FilterJob(hp.value, H.shape[0], ldh, vp.value, ldv, V.shape[1],
                           d.ctypes.data, mu1, alpha, beta)
    mv = ctypes.c_int64(0)
    _check(lib().chase_filter_fused(ctypes.cast(arr, _P), len(jobs), ctypes.byref(mv),
                                    _stream_ptr(stream)))
    del keep
    return mv.value


def lanczos(H, V0, k, stream=None):
    """(alpha[k, r], beta[k, r]) of k Lanczos steps from the columns of V0."""
    hp, ldh = _h_colmajor(H)
    N, r = V0.shape
    vp, ldv = _block(V0, "V0")
    al = np.zeros((k, r))
    be = np.zeros((k, r))
    _check(lib().chase_lanczos(hp, N, ldh, vp, ldv, r, k, al.ctypes.data_as(_P),
                               be.ctypes.data_as(_P), _stream_ptr(stream)))
    return al, be


def lanczos_bounds(al, be, N, ne):
    al = np.ascontiguousarray(al, dtype=np.float64)
    be = np.ascontiguousarray(be, dtype=np.float64)
    k, r = al.shape
    out = np.zeros(4)
    _check(lib().chase_lanczos_bounds(al.ctypes.data_as(_P), be.ctypes.data_as(_P),
                                      k, r, N, ne, out.ctypes.data_as(_P)))
    return tuple(float(x) for x in out)


def qr(V, nlocked=0, stream=None):
    N, n = V.shape
    vp, ldv = _block(V, "V")
    _check(lib().chase_qr(vp, N, ldv, n, nlocked, _stream_ptr(stream)))
    return V


def rayleigh_ritz(H, Q, stream=None, residuals=True):
    hp, ldh = _h_colmajor(H)
    N, n = Q.shape
    qp, ldq = _block(Q, "Q")
    th = np.zeros(n)
    rs = np.zeros(n) if residuals else None
    _check(lib().chase_rayleigh_ritz(hp, N, ldh, qp, ldq, n, th.ctypes.data_as(_P),
                                     rs.ctypes.data_as(_P) if residuals else None,
                                     _stream_ptr(stream)))
    return th, rs


def residuals(H, V, theta, stream=None):
    hp, ldh = _h_colmajor(H)
    N, n = V.shape
    vp, ldv = _block(V, "V")
    th = np.ascontiguousarray(theta, dtype=np.float64)
    rs = np.zeros(n)
    _check(lib().chase_residuals(hp, N, ldh, vp, ldv, n, th.ctypes.data_as(_P),
                                 rs.ctypes.data_as(_P), _stream_ptr(stream)))
    return rs


def heevj(G, stream=None):
    """Eigen-decomposition of a small Hermitian (n, n) row-major CUDA tensor."""
    torch = _torch()
    n = G.shape[0]
    gp, ldg = _block(G, "G")
    if ldg != n:
        raise ValueError("G must be contiguous")
    Y = torch.empty_like(G)
    w = np.zeros(n)
    _check(lib().chase_heevj(gp, n, w.ctypes.data_as(_P), _dptr(Y), _stream_ptr(stream)))
    return w, Y


def heevj_noalloc(G, Y=None, stream=None):
    """heevj through the allocation-free entry point (n <= 512): the library
    allocates nothing; Y (n, n) may be given to make the call allocation
    free on the Python side as well."""
    torch = _torch()
    n = G.shape[0]
    gp, ldg = _block(G, "G")
    if ldg != n:
        raise ValueError("G must be contiguous")
    if Y is None:
        Y = torch.empty_like(G)
    w = np.zeros(n)
    _check(lib().chase_heevj_noalloc(gp, n, w.ctypes.data_as(_P), _dptr(Y),
                                     _stream_ptr(stream)))
    return w, Y


def degrees(theta, resid, tol_abs, alpha, beta, degree_max, extra=2):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    rs = np.ascontiguousarray(resid, dtype=np.float64)
    out = np.zeros(th.size, dtype=np.int32)
    _check(lib().chase_degrees(th.ctypes.data_as(_P), rs.ctypes.data_as(_P), th.size,
                               tol_abs, alpha, beta, degree_max, extra,
                               out.ctypes.data_as(_P)))
    return out


# ------------------------------------------------------------ ingesting H

def ingest_rows(H, rows, r0, stream=None):
    """Rows [r0, r0 + len(rows)) of the lower triangle of H (row r has its
    columns 0..r in rows[r - r0]) into the column-major device matrix H, both
    triangles.  ``rows`` is a row-major complex128 block: a CUDA tensor, or
    host memory (a CPU tensor or numpy array; page-locked moves fastest),
    which is streamed to the device in chunks."""
    hp, ldh = _h_colmajor(H)
    N = H.shape[0]
    if isinstance(rows, np.ndarray):
        if rows.dtype != np.complex128 or rows.ndim != 2 or rows.strides[1] != 16 \
                or rows.strides[0] % 16:
            raise ValueError("rows must be a row-major complex128 array")
        ptr, ldr, on_dev = rows.ctypes.data, rows.strides[0] // 16, False
    else:
        torch = _torch()
        if rows.dtype != torch.complex128 or rows.dim() != 2 or rows.stride(1) != 1:
            raise ValueError("rows must be a row-major complex128 tensor")
        ptr, ldr, on_dev = rows.data_ptr(), rows.stride(0), rows.is_cuda
    fn = lib().chase_ingest_rows if on_dev else lib().chase_ingest_rows_host
    _check(fn(hp, N, ldh, ptr, ldr, r0, rows.shape[0], _stream_ptr(stream)))


def hermitian_complete(H, uplo="L", stream=None):
    """Complete the column-major device matrix H in place from its lower
    ('L') or upper ('U') triangle."""
    hp, ldh = _h_colmajor(H)
    _check(lib().chase_hermitian_complete(hp, H.shape[0], ldh, ord(uplo), _stream_ptr(stream)))


def nex_linear(nex_low, nex_high, e_low, e_high, e):
    """Supplement Eq. S2: nex interpolated linearly in the energy cutoff."""
    v = lib().chase_nex_linear(nex_low, nex_high, e_low, e_high, e)
    if v < 0:
        raise ChaseError(CHASE_EINVAL, last_error())
    return v


# ------------------------------------------------------------------ serving

FILL_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_void_p, ctypes.c_void_p)

SIGNATURES.update({
    "chase_server_create": (ctypes.c_void_p, [ctypes.c_size_t, _I32, ctypes.c_uint32]),
    "chase_server_set_aging": (ctypes.c_int, [_P, _D]),
    "chase_server_fusion_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_int64)]),
    "chase_server_submit": (ctypes.c_int, [_P, _P, ctypes.c_int, _I64, _I64, _I32, _I32, _D,
                                           _I32, ctypes.POINTER(ChaseOpts),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "chase_server_submit_fill": (ctypes.c_int, [_P, FILL_FN, _P, _I64, _I32, _I32, _D, _I32,
                                                ctypes.POINTER(ChaseOpts),
                                                ctypes.POINTER(ctypes.c_uint64)]),
    "chase_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, _P, _P, _P, _I64,
                                         ctypes.POINTER(ChaseInfo), _P]),
    "chase_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, _D]),
    "chase_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]),
    "chase_server_last_error": (ctypes.c_char_p, []),
    "chase_server_destroy": (None, [_P]),
})


@dataclass
class ServedResult:
    eigvals: np.ndarray
    resid: np.ndarray
    V: object                 # torch (N, nev) complex128, column-major memory
    status: int
    info: dict
    queued_s: float
    gpu_s: float
    latency_s: float


class Server:
    """Continuous-batching server (marshalling over chase_server_*).

    ``submit(H, ...)`` takes a device tensor held by the caller until it is
    polled (column-major, ldh == N); ``submit_fill(fill, N, ...)`` takes a
    callable fill(ptr, N, ld, stream_ptr) -> int run at admission on the
    slot's stream."""

    def __init__(self, budget_bytes=0, slots=4, fuse=False, shortest_first=False,
                 aging_s=None):
        L = lib()
        flags = (CHASE_SERVER_FUSE_FILTER if fuse else 0) | \
                (CHASE_SERVER_SHORTEST_FIRST if shortest_first else 0)
        self._s = L.chase_server_create(int(budget_bytes), int(slots), flags)
        if not self._s:
            msg = L.chase_server_last_error()
            raise ChaseError(CHASE_EINTERNAL, msg.decode() if msg else "create failed")
        if aging_s is not None:
            _check(L.chase_server_set_aging(self._s, float(aging_s)))
        self._keep = {}      # ticket -> objects kept alive (tensors, callbacks)
        self._shape = {}     # ticket -> (N, nev)

    def _err(self):
        msg = lib().chase_server_last_error()
        return msg.decode() if msg else ""

    def submit(self, H, nev, nex, tol=1e-10, degree_max=20, **opt_kw):
        hp, ldh, conj = _h_layout(H)
        if conj:
            raise ValueError("server requests take H column-major (strides (1, N))")
        N = H.shape[0]
        o = default_opts(**opt_kw)
        t = ctypes.c_uint64(0)
        # The server reads H on a stream of its own, not ordered after the
        # caller's: the work that produced H must be complete first.
        _torch().cuda.current_stream(H.device).synchronize()
        st = lib().chase_server_submit(self._s, hp, 1, N, ldh, nev, nex, tol, degree_max,
                                       ctypes.byref(o), ctypes.byref(t))
        if st != CHASE_OK:
            raise ChaseError(st, self._err())
        self._keep[t.value] = (H,)
        self._shape[t.value] = (N, nev)
        return t.value

    def submit_fill(self, fill, N, nev, nex, tol=1e-10, degree_max=20, **opt_kw):
        def _cb(ptr, n, ld, user, stream):
            try:
                return int(fill(ptr, n, ld, stream))
            except Exception:  # noqa: BLE001 - reported as a status to C
                return 1
        cb = FILL_FN(_cb)
        o = default_opts(**opt_kw)
        t = ctypes.c_uint64(0)
        st = lib().chase_server_submit_fill(self._s, cb, None, N, nev, nex, tol, degree_max,
                                            ctypes.byref(o), ctypes.byref(t))
        if st != CHASE_OK:
            raise ChaseError(st, self._err())
        self._keep[t.value] = (cb,)
        self._shape[t.value] = (N, nev)
        return t.value

    def wait(self, ticket, timeout=-1.0):
        return lib().chase_server_wait(self._s, ticket, float(timeout)) == CHASE_OK

    def poll(self, ticket, allow_noconv=False):
        """ServedResult when done, None while pending."""
        torch = _torch()
        N, nev = self._shape[ticket]
        out = torch.empty((nev, N), dtype=torch.complex128, device="cuda")
        ev = np.zeros(nev)
        rs = np.zeros(nev)
        info = ChaseInfo()
        times = np.zeros(3)
        # The result is copied on the server's own stream: work still queued
        # on this stream may use the memory the allocator just handed out.
        torch.cuda.current_stream(out.device).synchronize()
        st = lib().chase_server_poll(self._s, ticket, ev.ctypes.data_as(_P),
                                     rs.ctypes.data_as(_P), _dptr(out), N,
                                     ctypes.byref(info), times.ctypes.data_as(_P))
        if st == CHASE_PENDING:
            return None
        self._keep.pop(ticket, None)
        self._shape.pop(ticket, None)
        if st not in ((CHASE_OK, CHASE_ENOCONV) if allow_noconv else (CHASE_OK,)):
            raise ChaseError(st, self._err())
        return ServedResult(ev, rs, out.t(), st, info.as_dict(), *map(float, times))

    def stats(self):
        a, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
        c, d, e = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        lib().chase_server_stats(self._s, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                 ctypes.byref(d), ctypes.byref(e))
        t, k = ctypes.c_int64(0), ctypes.c_int64(0)
        lib().chase_server_fusion_stats(self._s, ctypes.byref(t), ctypes.byref(k))
        return {"bytes_in_use": a.value, "peak_bytes": b.value, "running": c.value,
                "peak_running": d.value, "queued": e.value, "fused_ticks": t.value,
                "fused_steps": k.value}

    def close(self):
        if self._s:
            lib().chase_server_destroy(self._s)
            self._s = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
