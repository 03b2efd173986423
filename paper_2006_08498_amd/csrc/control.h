// Host-side control of the solver (see control.cpp).
#pragma once

#include <cstdint>

namespace chase {

struct Bounds {
    double mu1;    // smallest Ritz value over the runs
    double mu_ne;  // spectral-density estimate of lambda_ne
    double bsup;   // upper bound: largest Ritz value + last beta, max over runs
    double hnorm;  // largest |Ritz value|: ||H||_2 from below
};

// al, be: k x r row-major [step][run].
Bounds lanczos_bounds(const double *al, const double *be, int k, int r,
                      int64_t N, int ne);

// Convergence factor |rho| of Eq. S1 for eigenvalue lam on the interval
// with centre c and half-width e (1 inside the interval).
double rate(double lam, double c, double e);

// Largest degree: degree_max rounded down to even (at least 2), or 1 when
// degree_max is 1.
int degree_cap(int degree_max);

// Smallest even m >= 2 (plus extra) with rate^m >= res / tol_abs, capped;
// always 1 when degree_max is 1.
int degree_for(double res, double tol_abs, double lam, double c, double e,
               int degree_max, int extra);

// Supplement Eq. S2: nex interpolated linearly in the energy cutoff between
// (e_low, nex_low) and (e_high, nex_high), rounded half away from zero, at
// least 0.  Requires e_high > e_low.
int nex_linear(int nex_low, int nex_high, double e_low, double e_high, double e);

}  // namespace chase
