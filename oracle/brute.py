"""Exact eigenvalues of tiny Hermitian matrices (test infrastructure only).

For a Hermitian matrix with Gaussian-integer (or any rational) entries, the
number of eigenvalues below a rational x equals the number of negative
pivots of the LDL^H factorisation of A - xI (Sylvester's law of inertia),
computed here in exact rational arithmetic.  Bisection on that count
brackets every eigenvalue, with multiplicity, to any width.  Nothing here
shares arithmetic with the floating-point solvers it checks.
"""
from __future__ import annotations

from fractions import Fraction


def _to_frac_matrix(A):
    n = len(A)
    M = []
    for i in range(n):
        row = []
        for j in range(n):
            z = complex(A[i][j])
            row.append((Fraction(z.real), Fraction(z.imag)))
        M.append(row)
    return M


def count_below(M, x):
    """Number of eigenvalues < x (rational), or None on a zero pivot."""
    n = len(M)
    W = [[(re - (x if i == j else 0), im) for j, (re, im) in enumerate(row)]
         for i, row in enumerate(M)]
    neg = 0
    for k in range(n):
        d = W[k][k][0]
        if d == 0:
            return None
        if d < 0:
            neg += 1
        for i in range(k + 1, n):
            ar, ai = W[i][k]
            if ar == 0 and ai == 0:
                continue
            for j in range(k + 1, n):
                br, bi = W[j][k]
                # W[i][j] -= W[i][k] * conj(W[j][k]) / d
                pr = (ar * br + ai * bi) / d
                pi = (ai * br - ar * bi) / d
                cr, ci = W[i][j]
                W[i][j] = (cr - pr, ci - pi)
    return neg


def _count(M, x):
    c = count_below(M, x)
    shift = Fraction(1, 2 ** 80)
    while c is None:               # x hit an eigenvalue of a leading minor
        x -= shift
        shift /= 2
        c = count_below(M, x)
    return c


def eigenvalues(A, width=Fraction(1, 2 ** 52)):
    """All eigenvalues of the Hermitian A, ascending, each as the midpoint
    of a rational bracket of the given width (repeated per multiplicity)."""
    M = _to_frac_matrix(A)
    n = len(M)
    radius = max(abs(M[i][i][0]) + sum(
        abs(complex(float(M[i][j][0]), float(M[i][j][1])))
        for j in range(n) if j != i) for i in range(n))
    bound = Fraction(int(radius) + 2)
    lo, hi = -bound, bound
    out = []

    def rec(a, b, ca, cb):
        if cb == ca:
            return
        if b - a <= width:
            out.extend([(a + b) / 2] * (cb - ca))
            return
        m = (a + b) / 2
        cm = _count(M, m)
        rec(a, m, ca, cm)
        rec(m, b, cm, cb)

    rec(lo, hi, _count(M, lo), _count(M, hi))
    return [float(v) for v in out]
