"""The solver's intermediate steps in plain FP64 numpy (test infrastructure).

Each function is the step written out in the paper's order and notation:
the supplement lists ChASE's phases as Lanczos (spectral estimates),
Filter (Chebyshev, repeated HEMM), QR, RR (Rayleigh-Ritz with a dense
reduced eigensolve and a GEMM back-transform) and Resid (residuals,
deflation and locking); the main text says the filter is a Chebyshev
three-term recurrence expressed with BLAS-3 and that ChASE fixes the work
needed ahead of time (Sec. "Solving the BSE eigenvalue problem on massively
parallel architectures").  Where the paper only names a step, the published
ChASE method it cites fixes the details (Winkelmann, Springer, Di Napoli,
ACM TOMS 45(2), 2019; scaled filter of Zhou & Saad, SIAM J. Matrix Anal.
Appl. 29, 2007).  Every reading taken here is listed in the design notes.

No blocking, fusion or reordering beyond what the definitions state.
"""
from __future__ import annotations

import math

import numpy as np

from . import eig as _eig


# --------------------------------------------------------------------------
# Filter interval and convergence rate (supplement, Eq. S1)
# --------------------------------------------------------------------------

def interval(alpha, beta):
    """Centre c and half-width e of the damped interval [alpha, beta]
    (supplement, text around Eq. S1)."""
    return 0.5 * (alpha + beta), 0.5 * (beta - alpha)


def rho(lam, c, e):
    """|rho| of Eq. S1: max over the sign of |t +- sqrt(t^2 - 1)|,
    t = (lam - c) / e.  The symbol gamma of the printed formula is read as
    the eigenvalue whose rate is wanted (the tables evaluate it at
    lambda_nev).  For |t| < 1 both roots have modulus 1."""
    t = (lam - c) / e
    s = np.sqrt(complex(t * t - 1.0))
    return max(abs(t + s), abs(t - s))


# --------------------------------------------------------------------------
# Chebyshev filter (Filter phase)
# --------------------------------------------------------------------------

def chebyshev_T(m, x):
    """C_m(x): cos(m arccos x) on [-1, 1], cosh(m arccosh |x|) (times
    (-1)^m for x < -1) outside it."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.cosh(m * np.arccosh(np.abs(xo))) * np.where(
        xo < 0, (-1.0) ** m, 1.0)
    return out


def cheb_step(H, Y, X, a, b, g):
    """One step of the three-term recurrence as a fused HEMM:
    W = a H Y + b Y + g X (X may be None when g == 0)."""
    W = a * (H @ Y) + b * Y
    if X is not None and g != 0.0:
        W = W + g * X
    return W


def filter_coefficients(mu1, alpha, beta, m):
    """(a_s, b_s, g_s) for s = 1..m of the scaled filter on [alpha, beta]
    normalised at mu1:  e = (beta-alpha)/2, c = (beta+alpha)/2,
    sigma_1 = e/(mu1-c), tau = 2/sigma_1,
    Y_1 = (sigma_1/e)(H - cI) Y_0,
    sigma_{s} = 1/(tau - sigma_{s-1}),
    Y_s = (2 sigma_s/e)(H - cI) Y_{s-1} - sigma_{s-1} sigma_s Y_{s-2}."""
    c, e = interval(alpha, beta)
    sigma1 = e / (mu1 - c)
    tau = 2.0 / sigma1
    out = []
    sigma_prev = sigma1
    for s in range(1, m + 1):
        if s == 1:
            a = sigma1 / e
            out.append((a, -c * a, 0.0))
        else:
            sigma = 1.0 / (tau - sigma_prev)
            a = 2.0 * sigma / e
            out.append((a, -c * a, -sigma_prev * sigma))
            sigma_prev = sigma
    return out


def cheb_filter(H, V, degrees, mu1, alpha, beta):
    """Filter column j of V with degree degrees[j] (per-vector degrees):
    every column runs the same recurrence and stops at its own degree."""
    V = np.asarray(V, dtype=np.complex128)
    degrees = np.asarray(degrees, dtype=np.int64)
    mmax = int(degrees.max()) if degrees.size else 0
    coefs = filter_coefficients(mu1, alpha, beta, mmax)
    prev = V.copy()          # Y_{s-2}
    cur = V.copy()           # Y_{s-1}
    out = V.copy()
    for s in range(1, mmax + 1):
        a, b, g = coefs[s - 1]
        act = degrees >= s
        if not act.any():
            break
        X = prev[:, act] if s > 1 else None
        nxt = cheb_step(H, cur[:, act], X, a, b, g)
        prev[:, act] = cur[:, act]
        cur[:, act] = nxt
        done = degrees == s
        out[:, done] = cur[:, done]
    return out


# --------------------------------------------------------------------------
# Spectral estimates by Lanczos (Lanczos phase)
# --------------------------------------------------------------------------

def lanczos(H, V0, k):
    """k Lanczos steps from each column of V0 (runs are independent).
    Returns (alpha[k, r], beta[k, r]) where T = tridiag(alpha; beta[:-1])
    and beta[-1] is the norm of the last residual.  No re-orthogonalisation
    (the estimates only set the filter interval)."""
    V0 = np.asarray(V0, dtype=np.complex128)
    N, r = V0.shape
    al = np.zeros((k, r))
    be = np.zeros((k, r))
    for run in range(r):
        v = V0[:, run] / np.linalg.norm(V0[:, run])
        vprev = np.zeros(N, dtype=np.complex128)
        bprev = 0.0
        for j in range(k):
            w = H @ v
            a = float(np.real(np.vdot(v, w)))
            w = w - a * v - bprev * vprev
            b = float(np.linalg.norm(w))
            al[j, run] = a
            be[j, run] = b
            vprev = v
            v = w / b if b > 0.0 else np.zeros_like(w)
            bprev = b
    return al, be


def lanczos_bounds(al, be, N, ne):
    """Bounds from the Lanczos tridiagonals (one per run):
    mu1 = smallest Ritz value (estimate of lambda_1);
    b_sup = max over runs of (largest Ritz value + last beta), the upper
    bound beta of the filter interval (fixed afterwards, supplement);
    mu_ne = smallest Ritz value x with N * mean_runs(sum of weights of Ritz
    values <= x) >= ne, the spectral-density estimate of lambda_ne; the
    weights are the squared first components of the T eigenvectors;
    hnorm = max |Ritz value|, a lower estimate of ||H||_2.
    mu_ne is a heuristic: parity unpinned."""
    k, r = al.shape
    thetas, weights = [], []
    mu1, bsup, hnorm = np.inf, -np.inf, 0.0
    for run in range(r):
        th, Z = _eig.tridiag_eig(al[:, run], be[:-1, run])
        w = Z[0, :] ** 2
        thetas.append(th)
        weights.append(w / r)
        mu1 = min(mu1, th[0])
        bsup = max(bsup, th[-1] + abs(be[-1, run]))
        hnorm = max(hnorm, abs(th[0]), abs(th[-1]))
    th = np.concatenate(thetas)
    w = np.concatenate(weights)
    order = np.argsort(th, kind="stable")
    cum = np.cumsum(w[order]) * N
    hit = np.nonzero(cum >= ne)[0]
    mu_ne = th[order][hit[0]] if hit.size else th[order][-1]
    return float(mu1), float(mu_ne), float(bsup), float(hnorm)


# --------------------------------------------------------------------------
# Degrees (work fixed ahead of time)
# --------------------------------------------------------------------------

def degree_cap(degree_max):
    """Largest degree a vector may get: the largest even degree not above
    degree_max (degrees are even so that every column of a two-buffer
    recurrence ends in the same buffer), except that degree_max = 1 allows
    exactly one step per iteration."""
    if degree_max == 1:
        return 1
    return max(2, degree_max - degree_max % 2)


def degree(res, tol_abs, lam, c, e, degree_max, extra=2):
    """Filter degree for one vector: the number of steps after which a
    residual res shrinking by 1/rho per step reaches tol_abs,
    m = ceil(ln(res / tol_abs) / ln rho) + extra, clamped to
    [2, degree_cap] and rounded up to even.  With degree_max = 1 every
    vector gets one step."""
    cap = degree_cap(degree_max)
    if cap == 1:
        return 1
    if res <= tol_abs:
        return 2
    r = rho(lam, c, e)
    if r <= 1.0 + 1e-12:
        return cap
    m = math.ceil(math.log(res / tol_abs) / math.log(r)) + extra
    m = min(max(m, 2), cap)
    return m + (m % 2)


# --------------------------------------------------------------------------
# QR, Rayleigh-Ritz, residuals, locking
# --------------------------------------------------------------------------

def qr_orth(V):
    """Orthonormal factor Q of V = Q R with diag(R) real positive (unique
    for full column rank); a library Householder QR is the step."""
    Q, R = np.linalg.qr(np.asarray(V, dtype=np.complex128))
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
    return Q * ph[None, :]


def orth_against(L, V):
    """Component of V orthogonal to the orthonormal columns of L
    (locked vectors are not modified by the QR phase)."""
    if L is None or L.shape[1] == 0:
        return V
    return V - L @ (L.conj().T @ V)


def rayleigh_ritz(H, Q):
    """G = Q^H H Q, G = Y diag(theta) Y^H, V = Q Y (theta ascending)."""
    G = Q.conj().T @ (H @ Q)
    G = 0.5 * (G + G.conj().T)
    theta, Y = _eig.eigh_lowest(G, G.shape[0])
    return theta, Q @ Y, Y


def residual_norms(H, V, theta):
    """r_j = ||H v_j - theta_j v_j||_2."""
    R = H @ V - V * np.asarray(theta)[None, :]
    return np.linalg.norm(R, axis=0)


def lock_count(res, tol_abs):
    """Length of the leading run of converged pairs (Ritz values ascending),
    so the locked set is always the lowest part of the spectrum."""
    n = 0
    for r in res:
        if r <= tol_abs:
            n += 1
        else:
            break
    return n


# --------------------------------------------------------------------------
# nex across a series of matrices (supplement, Eq. S2)
# --------------------------------------------------------------------------

def nex_linear(nex_low, nex_high, e_low, e_high, e):
    """nex for energy cutoff e on the straight line through (e_low, nex_low)
    and (e_high, nex_high), rounded to the nearest integer with halves away
    from zero, never below 0."""
    v = nex_low + (nex_high - nex_low) / (e_high - e_low) * (e - e_low)
    r = math.floor(abs(v) + 0.5)
    return max(0, r if v >= 0 else -r)


# --------------------------------------------------------------------------
# Ingesting H: the Hermitian matrix from one stored triangle (main text,
# Sec. "Matrix generation and the I/O challenge": the lower half is read,
# the upper half filled from the transposed parts)
# --------------------------------------------------------------------------

def hermitian_from_triangle(A, lower=True):
    """The Hermitian matrix whose stored triangle (lower or upper, diagonal
    included) is A's: each element of the other strict triangle is the
    conjugate of its mirror, and the diagonal keeps its real part.  Written
    element by element so that every value is a copy (or a sign flip) of
    A's, bit for bit."""
    A = np.asarray(A, dtype=np.complex128)
    N = A.shape[0]
    C = np.empty((N, N), dtype=np.complex128)
    i, j = np.tril_indices(N, -1)          # i > j
    if lower:
        C[i, j] = A[i, j]
        C[j, i] = np.conj(A[i, j])
    else:
        C[j, i] = A[j, i]
        C[i, j] = np.conj(A[j, i])
    d = np.arange(N)
    C[d, d] = A[d, d].real.astype(np.complex128)
    return C
