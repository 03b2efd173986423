// Host-side control of the solver (scalars only; no matrix ever visits the
// host): spectral bounds from the Lanczos tridiagonals, the filter interval,
// per-vector convergence rates (supplement, Eq. S1) and filter degrees.
#include "control.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace chase {

// Cyclic Jacobi on a small real symmetric matrix (row-major, n x n):
// eigenvalues in w (unsorted), eigenvectors as columns of Z.
static void sym_jacobi(std::vector<double> &A, int n, std::vector<double> &w,
                       std::vector<double> &Zm) {
    Zm.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Zm[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = A[(size_t)i * n + j] * A[(size_t)i * n + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
                for (int k = 0; k < n; ++k) {   // Z <- Z J
                    const double zkp = Zm[(size_t)k * n + p], zkq = Zm[(size_t)k * n + q];
                    Zm[(size_t)k * n + p] = c * zkp - s * zkq;
                    Zm[(size_t)k * n + q] = s * zkp + c * zkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

Bounds lanczos_bounds(const double *al, const double *be, int k, int r,
                      int64_t N, int ne) {
    Bounds b{};
    b.mu1 = INFINITY;
    b.bsup = -INFINITY;
    b.hnorm = 0.0;
    std::vector<double> th, wt;
    for (int run = 0; run < r; ++run) {
        std::vector<double> T((size_t)k * k, 0.0), w, Zm;
        for (int j = 0; j < k; ++j) {
            T[(size_t)j * k + j] = al[(size_t)j * r + run];
            if (j + 1 < k) {
                const double bj = be[(size_t)j * r + run];
                T[(size_t)j * k + j + 1] = T[(size_t)(j + 1) * k + j] = bj;
            }
        }
        sym_jacobi(T, k, w, Zm);
        double tmin = INFINITY, tmax = -INFINITY;
        for (int l = 0; l < k; ++l) {
            tmin = std::min(tmin, w[l]);
            tmax = std::max(tmax, w[l]);
            th.push_back(w[l]);
            wt.push_back(Zm[l] * Zm[l] / r);   // squared first component
        }
        b.mu1 = std::min(b.mu1, tmin);
        b.bsup = std::max(b.bsup, tmax + std::fabs(be[(size_t)(k - 1) * r + run]));
        b.hnorm = std::max(b.hnorm, std::max(std::fabs(tmin), std::fabs(tmax)));
    }
    std::vector<size_t> order(th.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t c) { return th[a] < th[c]; });
    double cum = 0.0;
    b.mu_ne = th[order.back()];
    for (size_t idx : order) {
        cum += wt[idx];
        if (cum * (double)N >= (double)ne) {
            b.mu_ne = th[idx];
            break;
        }
    }
    return b;
}

double rate(double lam, double c, double e) {
    const double t = (lam - c) / e;
    if (std::fabs(t) <= 1.0) return 1.0;
    const double a = std::fabs(t);
    return a + std::sqrt(a * a - 1.0);
}

// Even degrees leave every column of the two-buffer recurrence in the same
// buffer; degree_max = 1 is the one exception (one step for every vector).
int degree_cap(int degree_max) {
    return degree_max == 1 ? 1 : std::max(2, degree_max - degree_max % 2);
}

int degree_for(double res, double tol_abs, double lam, double c, double e,
               int degree_max, int extra) {
    const int cap = degree_cap(degree_max);
    if (cap == 1) return 1;
    if (res <= tol_abs) return 2;
    const double r = rate(lam, c, e);
    if (!(r > 1.0 + 1e-12)) return cap;
    const double m = std::ceil(std::log(res / tol_abs) / std::log(r)) + extra;
    int d = (int)std::min<double>(std::max<double>(m, 2.0), (double)cap);
    return d + (d % 2);   // cap is even, so this stays <= cap
}

int nex_linear(int nex_low, int nex_high, double e_low, double e_high, double e) {
    const double slope = (double)(nex_high - nex_low) / (e_high - e_low);
    const double v = std::round((double)nex_low + slope * (e - e_low));
    return (int)std::max(0.0, std::min(v, 2147483647.0));
}

}  // namespace chase
