/*
 * Oracle (test infrastructure only): the lowest nev eigenpairs of a dense
 * complex Hermitian matrix, in FP64, on the host.
 *
 * Only the test suite, the package's smoke check and the benchmark's CPU
 * baseline leg load this library.  It shares no code with the HIP path.
 *
 * What it computes is the plain definition of the eigensolver's result: the
 * nev algebraically smallest eigenvalues of H with orthonormal eigenvectors
 * (the paper seeks the low-lying excitonic eigenpairs, full eigenpairs and
 * not only eigenvalues; Sec. "Solving the BSE eigenvalue problem on
 * massively parallel architectures").  It is reached the textbook "direct"
 * way that section contrasts ChASE with: reduce H to tridiagonal form, then
 * iterate on the tridiagonal (Golub & Van Loan, Matrix Computations, 4th
 * ed., Sec. 8.3: Householder tridiagonalisation, Alg. 8.3.1; implicit
 * symmetric QR step with Wilkinson shift, Alg. 8.3.2; symmetric QR
 * algorithm, Alg. 8.3.3).
 *
 * Steps:
 *   1. A <- lower triangle of H, mirrored (the paper's reader reads only the
 *      lower half of H).
 *   2. For k = 0..N-3 a Householder reflector P_k = I - tau u u^H maps
 *      A[k+1:, k] onto a multiple of e_1; A <- P_k A P_k on the trailing
 *      block.  The result is a Hermitian tridiagonal T with real diagonal d
 *      and complex sub-diagonal f.
 *   3. T = D S D^H with D = diag(delta), delta_0 = 1,
 *      delta_{j+1} = delta_j f_j / |f_j|, and S real symmetric with
 *      sub-diagonal |f_j|.
 *   4. Implicit symmetric QR with Wilkinson shift on S, rotations
 *      accumulated into Z (S = Z Lambda Z^T).
 *   5. The nev smallest eigenvalues (ascending; ties keep index order).
 *   6. v = P_0 P_1 ... P_{N-3} D z for each chosen column z of Z.
 *   7. Phase: the entry of largest modulus (lowest index on ties) is made
 *      real and positive.
 *
 * Built with -ffp-contract=off (no fused multiply-add) and
 * -fcx-limited-range (plain complex product formula).
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 2, ORACLE_ENOCONV = 3 };

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Step 4: implicit symmetric QR (Wilkinson shift) on the real symmetric
 * tridiagonal with diagonal d[0..n-1] and off-diagonal e[0..n-2].
 * On return d holds the eigenvalues (unsorted).  If Z is not NULL it is an
 * n x n row-major matrix that is multiplied on the right by every rotation
 * (initialise it to the identity to get the eigenvectors as its columns).
 * Returns 0, or ORACLE_ENOCONV after 30 n QR steps.
 */
int oracle_tridiag_qr(int64_t n, double *d, double *e, double *Z, int nthreads)
{
    if (n <= 1) return ORACLE_OK;
    set_threads(nthreads);
    const double eps = DBL_EPSILON * 0.5; /* unit roundoff 2^-53 */
    double *cs = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    if (!cs) return ORACLE_ENOMEM;
    int64_t steps = 0, max_steps = 30 * n;
    int64_t hi = n - 1;
    while (hi > 0) {
        /* Deflate negligible couplings. */
        for (int64_t i = 0; i < hi; ++i)
            if (fabs(e[i]) <= eps * (fabs(d[i]) + fabs(d[i + 1]))) e[i] = 0.0;
        /* Shrink hi past the trailing diagonal part. */
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        /* The unreduced block is [lo, hi]. */
        int64_t lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++steps > max_steps) { free(cs); return ORACLE_ENOCONV; }

        /* Wilkinson shift from the trailing 2 x 2 block. */
        double dd = 0.5 * (d[hi - 1] - d[hi]);
        double b2 = e[hi - 1] * e[hi - 1];
        double sg = dd >= 0.0 ? 1.0 : -1.0;
        double mu = d[hi] - b2 / (dd + sg * sqrt(dd * dd + b2));

        double x = d[lo] - mu, z = e[lo];
        double bulge = 0.0;
        for (int64_t k = lo; k < hi; ++k) {
            if (k > lo) { x = e[k - 1]; z = bulge; }
            double r = hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) { c = x / r; s = z / r; }
            if (k > lo) e[k - 1] = r;
            /* T <- R T R^T with R = [[c, s], [-s, c]] in plane (k, k+1). */
            double a = d[k], b = e[k], dn = d[k + 1];
            d[k] = c * c * a + 2.0 * c * s * b + s * s * dn;
            d[k + 1] = s * s * a - 2.0 * c * s * b + c * c * dn;
            e[k] = (c * c - s * s) * b + c * s * (dn - a);
            if (k + 1 < hi) {
                bulge = s * e[k + 1];
                e[k + 1] = c * e[k + 1];
            }
            cs[2 * (k - lo)] = c;
            cs[2 * (k - lo) + 1] = s;
        }
        if (Z) {
            /* Z <- Z R^T for every rotation of this step, row by row. */
            int64_t nrot = hi - lo;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                double *zr = Z + i * n;
                for (int64_t t = 0; t < nrot; ++t) {
                    int64_t k = lo + t;
                    double c = cs[2 * t], s = cs[2 * t + 1];
                    double zk = zr[k], zk1 = zr[k + 1];
                    zr[k] = c * zk + s * zk1;
                    zr[k + 1] = -s * zk + c * zk1;
                }
            }
        }
    }
    free(cs);
    return ORACLE_OK;
}

/* Ascending order of w[0..n-1]; equal values keep index order. */
static const double *g_sort_keys;
static int cmp_idx(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    double wa = g_sort_keys[a], wb = g_sort_keys[b];
    if (wa < wb) return -1;
    if (wa > wb) return 1;
    return (a > b) - (a < b);
}

/* Steps 1-2: returns d (n), f (n-1), reflectors U (column k holds u_k in
 * rows k+1..n-1, column-major n x n) and tau (n). */
static int householder_tridiag(int64_t n, zc *A, double *d, zc *f, zc *U, double *tau)
{
    zc *p = (zc *)malloc(sizeof(zc) * (size_t)n);
    zc *w = (zc *)malloc(sizeof(zc) * (size_t)n);
    if (!p || !w) { free(p); free(w); return ORACLE_ENOMEM; }
    for (int64_t k = 0; k + 2 < n; ++k) {
        int64_t m = n - k - 1;              /* length of x = A[k+1:, k] */
        zc *x = A + (k + 1) + k * n;
        zc *u = U + (k + 1) + k * n;
        double tail = 0.0;                  /* sum |x_i|^2, i >= 1 */
        for (int64_t i = 1; i < m; ++i) tail += creal(x[i] * conj(x[i]));
        if (tail == 0.0) {                  /* already tridiagonal here */
            tau[k] = 0.0;
            d[k] = creal(A[k + k * n]);
            f[k] = x[0];
            continue;
        }
        double x0a = cabs(x[0]);
        double alpha = sqrt(x0a * x0a + tail);
        zc phase = x0a == 0.0 ? 1.0 : x[0] / x0a;
        for (int64_t i = 0; i < m; ++i) u[i] = x[i];
        u[0] = x[0] + phase * alpha;
        double uu = 0.0;
        for (int64_t i = 0; i < m; ++i) uu += creal(u[i] * conj(u[i]));
        double t = 2.0 / uu;
        tau[k] = t;
        d[k] = creal(A[k + k * n]);
        f[k] = -phase * alpha;              /* P x = -phase * alpha * e_1 */

        /* p = t * A22 u, using A22 u = A22^H u: p_i = conj(col_i) . u */
        zc *A22 = A + (k + 1) + (k + 1) * n;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            const zc *col = A22 + i * n;
            zc s = 0.0;
            for (int64_t j = 0; j < m; ++j) s += conj(col[j]) * u[j];
            p[i] = t * s;
        }
        /* K = t (u^H p) / 2 (real), w = p - K u */
        zc up = 0.0;
        for (int64_t i = 0; i < m; ++i) up += conj(u[i]) * p[i];
        double K = 0.5 * t * creal(up);
        for (int64_t i = 0; i < m; ++i) w[i] = p[i] - K * u[i];
        /* A22 <- A22 - u w^H - w u^H */
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < m; ++j) {
            zc *col = A22 + j * n;
            zc cw = conj(w[j]), cu = conj(u[j]);
            for (int64_t i = 0; i < m; ++i) col[i] -= u[i] * cw + w[i] * cu;
        }
    }
    if (n >= 2) {
        d[n - 2] = creal(A[(n - 2) + (n - 2) * n]);
        f[n - 2] = A[(n - 1) + (n - 2) * n];
        tau[n - 2] = 0.0;
    }
    d[n - 1] = creal(A[(n - 1) + (n - 1) * n]);
    if (n >= 1) tau[n - 1] = 0.0;
    free(p);
    free(w);
    return ORACLE_OK;
}

/*
 * The nev smallest eigenpairs of the Hermitian H (complex128 interleaved,
 * column-major, leading dimension ldh >= N; only the lower triangle is
 * read).  w: nev doubles, ascending.  V: N x nev complex128, column-major,
 * leading dimension N, or NULL for eigenvalues only (the O(N^3) rotation
 * accumulation is then skipped).  nthreads <= 0 keeps the OpenMP default.
 */
int oracle_eigh_lowest(int64_t N, const double *H, int64_t ldh, int32_t nev,
                       double *w, double *V, int nthreads)
{
    if (N < 1 || ldh < N || nev < 1 || nev > N || !H || !w) return ORACLE_EINVAL;
    set_threads(nthreads);
    size_t n = (size_t)N;
    zc *A = (zc *)malloc(sizeof(zc) * n * n);
    zc *U = (zc *)calloc(n * n, sizeof(zc));
    double *d = (double *)malloc(sizeof(double) * n);
    zc *f = (zc *)malloc(sizeof(zc) * n);
    double *e = (double *)malloc(sizeof(double) * n);
    double *tau = (double *)malloc(sizeof(double) * n);
    zc *delta = (zc *)malloc(sizeof(zc) * n);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * n);
    double *Z = NULL;
    int st = ORACLE_OK;
    if (!A || !U || !d || !f || !e || !tau || !delta || !idx) { st = ORACLE_ENOMEM; goto out; }

    /* Step 1: lower triangle, mirrored; diagonal taken as real. */
    const zc *Hz = (const zc *)H;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        for (int64_t i = j; i < N; ++i) {
            zc h = Hz[i + j * ldh];
            if (i == j) h = creal(h);
            A[i + j * N] = h;
            A[j + i * N] = conj(h);
        }
    }
    /* Step 2. */
    st = householder_tridiag(N, A, d, f, U, tau);
    if (st) goto out;

    /* Step 3: D = diag(delta), S off-diagonal |f_j|. */
    delta[0] = 1.0;
    for (int64_t j = 0; j + 1 < N; ++j) {
        double af = cabs(f[j]);
        e[j] = af;
        delta[j + 1] = af == 0.0 ? delta[j] : delta[j] * (f[j] / af);
    }

    /* Step 4. */
    if (V) {
        Z = (double *)calloc(n * n, sizeof(double));
        if (!Z) { st = ORACLE_ENOMEM; goto out; }
        for (int64_t i = 0; i < N; ++i) Z[i * N + i] = 1.0;
    }
    st = oracle_tridiag_qr(N, d, e, Z, nthreads);
    if (st) goto out;

    /* Step 5. */
    for (int64_t i = 0; i < N; ++i) idx[i] = i;
    g_sort_keys = d;
    qsort(idx, n, sizeof(int64_t), cmp_idx);
    for (int32_t j = 0; j < nev; ++j) w[j] = d[idx[j]];
    if (!V) goto out;

    /* Steps 6-7, one eigenvector per iteration. */
    zc *Vz = (zc *)V;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < nev; ++j) {
        zc *v = Vz + (size_t)j * n;
        int64_t c = idx[j];
        for (int64_t i = 0; i < N; ++i) v[i] = delta[i] * Z[i * N + c];
        for (int64_t k = N - 3; k >= 0; --k) {
            if (tau[k] == 0.0) continue;
            const zc *u = U + (k + 1) + k * N;
            zc *y = v + (k + 1);
            int64_t m = N - k - 1;
            zc s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += conj(u[i]) * y[i];
            s *= tau[k];
            for (int64_t i = 0; i < m; ++i) y[i] -= s * u[i];
        }
        int64_t imax = 0;
        double amax = -1.0;
        for (int64_t i = 0; i < N; ++i) {
            double a = cabs(v[i]);
            if (a > amax) { amax = a; imax = i; }
        }
        zc ph = amax > 0.0 ? conj(v[imax]) / amax : 1.0;
        for (int64_t i = 0; i < N; ++i) v[i] *= ph;
        v[imax] = creal(v[imax]);
    }
out:
    free(A); free(U); free(d); free(f); free(e); free(tau); free(delta); free(idx); free(Z);
    return st;
}
