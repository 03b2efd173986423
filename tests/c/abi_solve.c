/*
 * A plain C consumer of the library's C ABI (no Python, no C++): the lowest
 * eigenpairs of a dense Hermitian matrix with a known spectrum.
 *
 * H = P D P with D = diag(1 + 5 i / N) and P = I - 2 v v^H a Householder
 * reflector (v a unit vector with complex entries), so H is dense and
 * Hermitian and its eigenvalues are exactly the entries of D.  Only the lower
 * triangle is uploaded; chase_hermitian_complete fills the upper one on the
 * device, then chase_solve_ex returns the nev lowest pairs.  The program
 * checks the eigenvalues against D, and every pair's residual and the
 * orthonormality of the vectors on the host in FP64.  Exit status 0 and the
 * last line "ok" mean success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "chase_mi355x.h"

#define CHECK_HIP(x)                                                            \
    do {                                                                        \
        hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) {                                                 \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));      \
            return 2;                                                           \
        }                                                                       \
    } while (0)

int main(void) {
    const int64_t N = 500;
    const int32_t nev = 10, nex = 6, degree_max = 20;
    const double tol = 1e-10;
    chase_z *H = calloc((size_t)(N * N), sizeof(chase_z));
    chase_z *Hlow = calloc((size_t)(N * N), sizeof(chase_z));
    chase_z *V = calloc((size_t)(N * nev), sizeof(chase_z));
    double *D = malloc((size_t)N * sizeof(double)), *vr = malloc((size_t)N * sizeof(double)),
           *vi = malloc((size_t)N * sizeof(double));
    double eig[10], res[10];
    if (!H || !Hlow || !V || !D || !vr || !vi) return 2;

    /* v: a fixed unit vector with complex entries; s = v^H D v. */
    double nrm = 0.0, s = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        D[i] = 1.0 + 5.0 * (double)i / (double)N;
        vr[i] = cos(0.37 * (double)i) + 0.5;
        vi[i] = sin(0.91 * (double)i);
        nrm += vr[i] * vr[i] + vi[i] * vi[i];
    }
    nrm = sqrt(nrm);
    for (int64_t i = 0; i < N; ++i) {
        vr[i] /= nrm;
        vi[i] /= nrm;
        s += D[i] * (vr[i] * vr[i] + vi[i] * vi[i]);
    }
    /* H(i, j) = D_i delta_ij + v_i conj(v_j) (4 s - 2 D_i - 2 D_j): the lower
     * triangle computed, the upper one its conjugate (column-major). */
    for (int64_t j = 0; j < N; ++j)
        for (int64_t i = j; i < N; ++i) {
            const double f = 4.0 * s - 2.0 * D[i] - 2.0 * D[j];
            chase_z h;
            h.re = (vr[i] * vr[j] + vi[i] * vi[j]) * f;
            h.im = (vi[i] * vr[j] - vr[i] * vi[j]) * f;
            if (i == j) {
                h.re += D[i];
                h.im = 0.0;
            }
            H[i + j * N] = h;
            Hlow[i + j * N] = h;
            if (i != j) {
                H[j + i * N].re = h.re;
                H[j + i * N].im = -h.im;
            }
        }

    chase_z *dH = NULL, *dV = NULL;
    CHECK_HIP(hipMalloc((void **)&dH, (size_t)(N * N) * sizeof(chase_z)));
    CHECK_HIP(hipMalloc((void **)&dV, (size_t)(N * nev) * sizeof(chase_z)));
    CHECK_HIP(hipMemcpy(dH, Hlow, (size_t)(N * N) * sizeof(chase_z), hipMemcpyHostToDevice));
    if (chase_hermitian_complete(dH, N, N, 'L', NULL) != CHASE_OK) {
        fprintf(stderr, "chase_hermitian_complete: %s\n", chase_last_error());
        return 1;
    }
    chase_opts o;
    chase_info info;
    chase_default_opts(&o);
    int st = chase_solve_ex(dH, N, N, nev, nex, tol, degree_max, eig, res, dV, N, NULL, 0,
                            NULL, &o, &info);
    if (st != CHASE_OK) {
        fprintf(stderr, "chase_solve_ex: status %d: %s\n", st, chase_last_error());
        return 1;
    }
    CHECK_HIP(hipMemcpy(V, dV, (size_t)(N * nev) * sizeof(chase_z), hipMemcpyDeviceToHost));
    CHECK_HIP(hipFree(dH));
    CHECK_HIP(hipFree(dV));

    /* ||H||_2 = max |D| = D[N - 1]; D is ascending, so the wanted
     * eigenvalues are D[0 .. nev-1]. */
    const double hn = D[N - 1];
    double worst_eig = 0.0, worst_res = 0.0, worst_orth = 0.0;
    for (int j = 0; j < nev; ++j) {
        worst_eig = fmax(worst_eig, fabs(eig[j] - D[j]) / fabs(D[j]));
        double rr = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double ar = 0.0, ai = 0.0;
            for (int64_t k = 0; k < N; ++k) {
                const chase_z h = H[i + k * N], x = V[k + (int64_t)j * N];
                ar += h.re * x.re - h.im * x.im;
                ai += h.re * x.im + h.im * x.re;
            }
            ar -= eig[j] * V[i + (int64_t)j * N].re;
            ai -= eig[j] * V[i + (int64_t)j * N].im;
            rr += ar * ar + ai * ai;
        }
        worst_res = fmax(worst_res, sqrt(rr) / hn);
        for (int l = 0; l < nev; ++l) {
            double gr = 0.0, gi = 0.0;
            for (int64_t i = 0; i < N; ++i) {
                const chase_z a = V[i + (int64_t)j * N], b = V[i + (int64_t)l * N];
                gr += a.re * b.re + a.im * b.im;
                gi += a.re * b.im - a.im * b.re;
            }
            worst_orth = fmax(worst_orth, hypot(gr - (j == l ? 1.0 : 0.0), gi));
        }
    }
    printf("N=%lld nev=%d iterations=%d matvecs=%lld: max rel eigenvalue error %.2e, "
           "max residual %.2e, orthogonality %.2e\n",
           (long long)N, nev, info.iterations, (long long)info.matvecs_filter, worst_eig,
           worst_res, worst_orth);
    if (!(worst_eig <= 1e-10 && worst_res <= 1e-10 && worst_orth <= 1e-12)) {
        printf("FAILED\n");
        return 1;
    }
    printf("ok\n");
    free(H);
    free(Hlow);
    free(V);
    free(D);
    free(vr);
    free(vi);
    return 0;
}
