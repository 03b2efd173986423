// Small dense kernels on the reduced matrices (order n <= 1024, typically
// nev + nex <= 400), all on the device so the solver never round-trips a
// matrix through the host:
//  * the CholeskyQR factor (QR phase): D = diag(G)^{-1/2}, Cholesky of
//    D G D + shift I, and B = D L^{-H} so that V <- V B orthonormalises;
//  * cyclic two-sided Jacobi for the reduced Hermitian eigenproblem of the
//    Rayleigh-Ritz phase (round-robin pairing, one launch per round, every
//    2 x 2 block updated independently: A' = J_a^H A J_b);
//  * ordering of the eigenpairs, Hermitian symmetrisation.
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace chase {
namespace {

__device__ __forceinline__ Z zmul(Z a, Z b) {
    return Z{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ Z zconj(Z a) { return Z{a.x, -a.y}; }
__device__ __forceinline__ Z zadd(Z a, Z b) { return Z{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Z zsub(Z a, Z b) { return Z{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ Z zscale(Z a, double s) { return Z{a.x * s, a.y * s}; }

// ---------------------------------------------------------- CholeskyQR
// CholeskyQR factor, one workgroup of 8 waves: G (n x n Hermitian,
// row-major, n <= 1024, not modified) -> B = D L^{-H} (upper triangular,
// row-major) with L the lower Cholesky factor of W = D G D + shift I and
// D = diag(G)^{-1/2}, so that V <- V B orthonormalises.  *info = 0, or
// j + 1 for the first non-positive (or non-finite) pivot j (then B is not
// written).
//
// Blocked in 16 x 16 complex blocks (nt = ceil(n / 16) per side; W is
// padded with the identity to 16 nt, which leaves L and L^{-1} padded with
// the identity), right-looking:
//  * step k: the diagonal block W_kk is factored in LDS by one wave and its
//    inverse formed by column-parallel forward substitution (no workgroup
//    barrier inside; three per block column in all); the panel L_ik = W_ik L_kk^{-H} (i > k) and the trailing
//    update W_ij -= L_ik L_jk^H (k < j <= i) are 16 x 16 x 16 complex
//    products on FP64 MFMA, one block per wave at a time;
//  * then X = L^{-1} by block rows: X_ii = L_ii^{-1} and, for k < i,
//    X_ik = -L_ii^{-1} sum_{j=k}^{i-1} L_ij X_jk (the sum's result feeds the
//    second product straight from the accumulator registers).
// W, X, the diagonal blocks' inverses and D live in `work`
// (chol_work_elems(n)), L2-resident at these orders.

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += A B for 16 x 16 complex blocks, K = 16, in the layout of the FP64
// 16x16x4 MFMA: lane (r, q) = (lane % 16, lane / 16) supplies A[r][4s + q]
// and B[4s + q][r] at k step s, and register v of its accumulators holds
// C[q + 4v][r].
template <class FA, class FB>
__device__ __forceinline__ void zblock_mac(v4d &cr, v4d &ci, FA a_at, FB b_at) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const Z a = a_at(s), b = b_at(s);
        cr = mfma64(a.x, b.x, cr);
        ci = mfma64(a.x, b.y, ci);
        cr = mfma64(-a.y, b.y, cr);
        ci = mfma64(a.y, b.x, ci);
    }
}

// 8 waves (2 per SIMD): room is left on the CU for other kernels (a
// 16-wave workgroup of this register size needs a whole idle CU, which a
// busy GPU rarely has).
constexpr int kCholThreads = 512;

size_t chol_np(int n) { return (size_t)(n + 15) / 16 * 16; }

// Orders the LDS accesses of one wave's lanes (no other wave is involved).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kCholThreads) void k_chol_blocked(const Z *__restrict__ G, int n,
                                                               double shift, Z *__restrict__ B,
                                                               Z *__restrict__ work,
                                                               int *info) {
    __shared__ Z dblk[16][17];   // diagonal block being factored (lower)
    __shared__ Z linv[16][17];   // its inverse
    __shared__ double ldg[16];   // its diagonal
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nwaves = kCholThreads / 64;
    const int r = lane & 15, q = lane >> 4;
    const int nt = (n + 15) / 16, np = 16 * nt;
    Z *W = work;                                  // np x np, row-major
    Z *X = W + (size_t)np * np;                   // np x np: L^{-1}
    Z *Li = X + (size_t)np * np;                  // nt blocks of 16 x 16
    double *dsc = reinterpret_cast<double *>(Li + (size_t)nt * 256);   // np

    if (t == 0) bad = 0x7fffffff;
    __syncthreads();
    for (int j = t; j < n; j += kCholThreads) {
        const double gjj = G[(int64_t)j * n + j].x;
        if (!(gjj > 0.0) || !isfinite(gjj)) atomicMin(&bad, j + 1);   // LDS atomic
        dsc[j] = gjj > 0.0 ? 1.0 / sqrt(gjj) : 0.0;
    }
    __syncthreads();
    if (bad != 0x7fffffff) {
        if (t == 0) *info = bad;
        return;
    }
    // W = D G D + shift I, padded with the identity.
    for (int64_t e = t; e < (int64_t)np * np; e += kCholThreads) {
        const int i = (int)(e / np), j = (int)(e - (int64_t)i * np);
        Z v{i == j ? 1.0 : 0.0, 0.0};
        if (i < n && j < n) {
            v = zscale(G[(int64_t)i * n + j], dsc[i] * dsc[j]);
            if (i == j) v = Z{v.x + shift, 0.0};
        }
        W[e] = v;
        X[e] = Z{0.0, 0.0};
    }
    __syncthreads();

    for (int k = 0; k < nt; ++k) {
        const int64_t kk0 = (int64_t)16 * k;
        // ---- diagonal block: Cholesky and inverse in LDS by wave 0 alone
        // (its lanes order their LDS accesses among themselves; the other
        // waves wait at the barrier below).
        if (wave == 0) {
            for (int e = lane; e < 256; e += 64) {
                const int i = e >> 4, m = e & 15;
                dblk[i][m] = m <= i ? W[(kk0 + i) * np + kk0 + m] : Z{0.0, 0.0};
            }
            wave_sync();
            for (int j = 0; j < 16; ++j) {
                const double piv = dblk[j][j].x;
                if (!(piv > 0.0) || !isfinite(piv)) {
                    if (lane == 0) bad = 16 * k + j + 1;
                    break;   // uniform across the wave: every lane read the same pivot
                }
                const double l = sqrt(piv), il = 1.0 / l;
                if (lane == 0) ldg[j] = l;
                if (lane > j && lane < 16) dblk[lane][j] = zscale(dblk[lane][j], il);
                wave_sync();
                for (int e = lane; e < 256; e += 64) {
                    const int i = e >> 4, m = e & 15;
                    if (m > j && m <= i)
                        dblk[i][m] = zsub(dblk[i][m], zmul(dblk[i][j], zconj(dblk[m][j])));
                }
                wave_sync();
            }
            wave_sync();
            if (bad == 0x7fffffff) {
                if (lane < 16) dblk[lane][lane] = Z{ldg[lane], 0.0};
                wave_sync();
                // Inverse, one column per lane (forward substitution).
                if (lane < 16) {
                    const int c = lane;
                    for (int i = 0; i < 16; ++i) {
                        Z acc{i == c ? 1.0 : 0.0, 0.0};
                        for (int m = c; m < i; ++m) acc = zsub(acc, zmul(dblk[i][m], linv[m][c]));
                        linv[i][c] = i < c ? Z{0.0, 0.0} : zscale(acc, 1.0 / ldg[i]);
                    }
                }
            }
        }
        __syncthreads();
        if (bad != 0x7fffffff) {
            if (t == 0) *info = bad;
            return;   // uniform: every thread reads the flag after the barrier
        }
        if (t < 256) {
            const int i = t >> 4, m = t & 15;
            Li[(int64_t)k * 256 + i * 16 + m] = linv[i][m];
            X[(kk0 + i) * np + kk0 + m] = linv[i][m];
        }
        // ---- panel: L_ik = W_ik L_kk^{-H}, i > k
        for (int i = k + 1 + wave; i < nt; i += nwaves) {
            const Z *Wi = W + (int64_t)16 * i * np + kk0;
            v4d cr{0, 0, 0, 0}, ci{0, 0, 0, 0};
            zblock_mac(cr, ci, [&](int s) { return Wi[(int64_t)r * np + 4 * s + q]; },
                       [&](int s) { return zconj(linv[r][4 * s + q]); });
            Z *Wo = W + (int64_t)16 * i * np + kk0;
#pragma unroll
            for (int v = 0; v < 4; ++v) Wo[(int64_t)(q + 4 * v) * np + r] = Z{cr[v], ci[v]};
        }
        __syncthreads();
        // ---- trailing update: W_ij -= L_ik L_jk^H, k < j <= i
        const int m = nt - k - 1;
        const int tiles = m * (m + 1) / 2;
        for (int tt = wave; tt < tiles; tt += nwaves) {
            int ii = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
            while (ii * (ii + 1) / 2 > tt) --ii;
            while ((ii + 1) * (ii + 2) / 2 <= tt) ++ii;
            const int jj = tt - ii * (ii + 1) / 2;
            const int i = k + 1 + ii, j = k + 1 + jj;
            Z *Wij = W + (int64_t)16 * i * np + 16 * j;
            const Z *Lik = W + (int64_t)16 * i * np + kk0;
            const Z *Ljk = W + (int64_t)16 * j * np + kk0;
            v4d cr, ci;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Z w = Wij[(int64_t)(q + 4 * v) * np + r];
                cr[v] = w.x;
                ci[v] = w.y;
            }
            zblock_mac(cr, ci,
                       [&](int s) {
                           const Z a = Lik[(int64_t)r * np + 4 * s + q];
                           return Z{-a.x, -a.y};
                       },
                       [&](int s) { return zconj(Ljk[(int64_t)r * np + 4 * s + q]); });
#pragma unroll
            for (int v = 0; v < 4; ++v) Wij[(int64_t)(q + 4 * v) * np + r] = Z{cr[v], ci[v]};
        }
        __syncthreads();
    }

    // ---- X = L^{-1} by block rows
    for (int i = 1; i < nt; ++i) {
        const Z *Lii = Li + (int64_t)i * 256;
        for (int k = wave; k < i; k += nwaves) {
            v4d cr{0, 0, 0, 0}, ci{0, 0, 0, 0};
            for (int j = k; j < i; ++j) {
                const Z *Lij = W + (int64_t)16 * i * np + 16 * j;
                const Z *Xjk = X + (int64_t)16 * j * np + 16 * k;
                zblock_mac(cr, ci, [&](int s) { return Lij[(int64_t)r * np + 4 * s + q]; },
                           [&](int s) { return Xjk[(int64_t)(4 * s + q) * np + r]; });
            }
            v4d xr{0, 0, 0, 0}, xi{0, 0, 0, 0};
            zblock_mac(xr, xi,
                       [&](int s) {
                           const Z a = Lii[r * 16 + 4 * s + q];
                           return Z{-a.x, -a.y};
                       },
                       [&](int s) { return Z{cr[s], ci[s]}; });
            Z *Xik = X + (int64_t)16 * i * np + 16 * k;
#pragma unroll
            for (int v = 0; v < 4; ++v) Xik[(int64_t)(q + 4 * v) * np + r] = Z{xr[v], xi[v]};
        }
        __syncthreads();
    }
    // ---- B = D X^H (upper triangular), row j, column i
    for (int64_t e = t; e < (int64_t)n * n; e += kCholThreads) {
        const int j = (int)(e / n), i = (int)(e - (int64_t)j * n);
        B[e] = i >= j ? zscale(zconj(X[(int64_t)i * np + j]), dsc[j]) : Z{0.0, 0.0};
    }
    if (t == 0) *info = 0;
}

// ---------------------------------------------------------- Jacobi
// Round-robin pairing of m (even) indices, round r, pair k.
__device__ __forceinline__ void rr_pair(int m, int r, int k, int &p, int &q) {
    int a, b;
    if (k == 0) {
        a = m - 1;
        b = r;
    } else {
        a = (r + k) % (m - 1);
        b = (r - k + (m - 1)) % (m - 1);
    }
    p = min(a, b);
    q = max(a, b);
}

// J = [[c, s], [-s e, c e]] with e = conj(a_pq)/|a_pq| diagonalises the
// 2 x 2 Hermitian [[a_pp, a_pq], [conj(a_pq), a_qq]] (complex phase then
// real symmetric Jacobi rotation, Golub & Van Loan Alg. 8.5.1).
struct Rot {
    double c, s;
    Z e;
    double dp, dq;   // resulting diagonal
    bool active;
};

__device__ Rot make_rot(const Z *A, int n, int p, int q) {
    Rot R{1.0, 0.0, Z{1.0, 0.0}, 0.0, 0.0, false};
    const double app = A[(int64_t)p * n + p].x;   // p < n always
    R.dp = app;
    if (q >= n) return R;      // phantom partner (n odd): identity
    const double aqq = A[(int64_t)q * n + q].x;
    const Z apq = A[(int64_t)p * n + q];
    const double x = sqrt(apq.x * apq.x + apq.y * apq.y);
    R.dp = app;
    R.dq = aqq;
    if (!(x > 1e-300) || x <= 1e-18 * (fabs(app) + fabs(aqq))) return R;
    R.e = Z{apq.x / x, -apq.y / x};
    const double tau = (aqq - app) / (2.0 * x);
    double t;
    if (fabs(tau) > 1e150) t = 0.5 / tau;
    else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    R.c = 1.0 / sqrt(1.0 + t * t);
    R.s = t * R.c;
    R.dp = app - t * x;
    R.dq = aqq + t * x;
    R.active = true;
    return R;
}

__global__ __launch_bounds__(256) void k_jacobi_round(
    const Z *__restrict__ A, Z *__restrict__ A2, const Z *__restrict__ V,
    Z *__restrict__ V2, int n, int m, int round) {
    const int h = m / 2;
    const int64_t nblk = (int64_t)h * h;
    const int64_t total = nblk + (int64_t)n * h;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nblk) {
            const int ka = (int)(t / h), kb = (int)(t - (int64_t)ka * h);
            int pa, qa, pb, qb;
            rr_pair(m, round, ka, pa, qa);
            rr_pair(m, round, kb, pb, qb);
            const Rot Ra = make_rot(A, n, pa, qa);
            const Rot Rb = make_rot(A, n, pb, qb);
            const bool qa_ok = qa < n, qb_ok = qb < n;
            if (ka == kb) {
                // Diagonal block: the rotation diagonalises it exactly.
                A2[(int64_t)pa * n + pa] = Z{Ra.dp, 0.0};
                if (qa_ok) {
                    A2[(int64_t)qa * n + qa] = Z{Ra.dq, 0.0};
                    A2[(int64_t)pa * n + qa] = Ra.active ? Z{0.0, 0.0} : A[(int64_t)pa * n + qa];
                    A2[(int64_t)qa * n + pa] = Ra.active ? Z{0.0, 0.0} : A[(int64_t)qa * n + pa];
                }
                continue;
            }
            const Z zero{0.0, 0.0};
            const Z m00 = A[(int64_t)pa * n + pb];
            const Z m01 = qb_ok ? A[(int64_t)pa * n + qb] : zero;
            const Z m10 = qa_ok ? A[(int64_t)qa * n + pb] : zero;
            const Z m11 = (qa_ok && qb_ok) ? A[(int64_t)qa * n + qb] : zero;
            // T = M J_b
            const Z j00b{Rb.c, 0.0}, j01b{Rb.s, 0.0};
            const Z j10b = zscale(Rb.e, -Rb.s), j11b = zscale(Rb.e, Rb.c);
            const Z t00 = zadd(zmul(m00, j00b), zmul(m01, j10b));
            const Z t01 = zadd(zmul(m00, j01b), zmul(m01, j11b));
            const Z t10 = zadd(zmul(m10, j00b), zmul(m11, j10b));
            const Z t11 = zadd(zmul(m10, j01b), zmul(m11, j11b));
            // A' = J_a^H T
            const Z c00{Ra.c, 0.0}, c10 = zconj(zscale(Ra.e, -Ra.s));
            const Z c01{Ra.s, 0.0}, c11 = zconj(zscale(Ra.e, Ra.c));
            A2[(int64_t)pa * n + pb] = zadd(zmul(c00, t00), zmul(c10, t10));
            if (qb_ok) A2[(int64_t)pa * n + qb] = zadd(zmul(c00, t01), zmul(c10, t11));
            if (qa_ok) A2[(int64_t)qa * n + pb] = zadd(zmul(c01, t00), zmul(c11, t10));
            if (qa_ok && qb_ok)
                A2[(int64_t)qa * n + qb] = zadd(zmul(c01, t01), zmul(c11, t11));
        } else {
            const int64_t u = t - nblk;
            const int i = (int)(u / h), kb = (int)(u - (int64_t)i * h);
            int pb, qb;
            rr_pair(m, round, kb, pb, qb);
            const Rot Rb = make_rot(A, n, pb, qb);
            const Z vp = V[(int64_t)i * n + pb];
            if (qb >= n) {
                V2[(int64_t)i * n + pb] = vp;
                continue;
            }
            const Z vq = V[(int64_t)i * n + qb];
            const Z j10b = zscale(Rb.e, -Rb.s), j11b = zscale(Rb.e, Rb.c);
            V2[(int64_t)i * n + pb] = zadd(zscale(vp, Rb.c), zmul(vq, j10b));
            V2[(int64_t)i * n + qb] = zadd(zscale(vp, Rb.s), zmul(vq, j11b));
        }
    }
}

// The whole cyclic Jacobi of a small reduced problem in one launch of one
// workgroup, with the convergence test (the host's: off <= 1e-15 tot, or
// off <= 1e-12 tot and no longer halving) on the device, so a solve's
// eigensolve is one launch instead of one per round (under concurrent
// solves each of those launches waits for room on the GPU).  Each round
// computes the m / 2 rotations, then applies them in place to every 2 x 2
// block (pa, qa) x (pb, qb) of A and to the pairs of columns of V (every
// block and column pair is owned by one thread, so no entry is read after
// another thread wrote it), and each sweep ends with the off-diagonal norm.
// Then w (ascending, ties by index) and Y[:, rank] = V[:, j].  *status =
// sweeps done, -1 if the cap was reached without convergence, -2 on a
// non-finite norm.  A and V (n x n row-major) live in LDS, up to
// kJacobiLds.  (The same sweeps with A and V in L2 for orders up to 320
// were measured and not kept: at n = 140 the one workgroup took 10 ms per
// eigensolve against 4 ms for the round launches of the sweep graphs.)
constexpr int kJacobiLds = 64;

__device__ __forceinline__ void jacobi_all_sweeps(const Z *__restrict__ A0, Z *As, Z *Vs,
                                                  Rot *rot, double (*red)[1024], int n,
                                                  int max_sweeps, double *__restrict__ w,
                                                  Z *__restrict__ Y, int *status) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int m = n + (n & 1), h = m / 2;
    for (int e = t; e < n * n; e += nt) {
        As[e] = A0[e];
        Vs[e] = Z{(e / n) == (e % n) ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    double prev = 1e300;
    int result = -1;
    for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
        for (int round = 0; round < m - 1; ++round) {
            for (int k = t; k < h; k += nt) {
                int p, q;
                rr_pair(m, round, k, p, q);
                rot[k] = make_rot(As, n, p, q);
            }
            __syncthreads();
            for (int e = t; e < h * h + n * h; e += nt) {
                if (e < h * h) {
                    const int ka = e / h, kb = e - ka * h;
                    int pa, qa, pb, qb;
                    rr_pair(m, round, ka, pa, qa);
                    rr_pair(m, round, kb, pb, qb);
                    const Rot Ra = rot[ka], Rb = rot[kb];
                    const bool qa_ok = qa < n, qb_ok = qb < n;
                    if (ka == kb) {
                        As[pa * n + pa] = Z{Ra.dp, 0.0};
                        if (qa_ok) {
                            As[qa * n + qa] = Z{Ra.dq, 0.0};
                            if (Ra.active) As[pa * n + qa] = As[qa * n + pa] = Z{0.0, 0.0};
                        }
                        continue;
                    }
                    const Z zero{0.0, 0.0};
                    const Z m00 = As[pa * n + pb];
                    const Z m01 = qb_ok ? As[pa * n + qb] : zero;
                    const Z m10 = qa_ok ? As[qa * n + pb] : zero;
                    const Z m11 = (qa_ok && qb_ok) ? As[qa * n + qb] : zero;
                    const Z j00b{Rb.c, 0.0}, j01b{Rb.s, 0.0};
                    const Z j10b = zscale(Rb.e, -Rb.s), j11b = zscale(Rb.e, Rb.c);
                    const Z t00 = zadd(zmul(m00, j00b), zmul(m01, j10b));
                    const Z t01 = zadd(zmul(m00, j01b), zmul(m01, j11b));
                    const Z t10 = zadd(zmul(m10, j00b), zmul(m11, j10b));
                    const Z t11 = zadd(zmul(m10, j01b), zmul(m11, j11b));
                    const Z c00{Ra.c, 0.0}, c10 = zconj(zscale(Ra.e, -Ra.s));
                    const Z c01{Ra.s, 0.0}, c11 = zconj(zscale(Ra.e, Ra.c));
                    As[pa * n + pb] = zadd(zmul(c00, t00), zmul(c10, t10));
                    if (qb_ok) As[pa * n + qb] = zadd(zmul(c00, t01), zmul(c10, t11));
                    if (qa_ok) As[qa * n + pb] = zadd(zmul(c01, t00), zmul(c11, t10));
                    if (qa_ok && qb_ok) As[qa * n + qb] = zadd(zmul(c01, t01), zmul(c11, t11));
                } else {
                    const int u = e - h * h;
                    const int i = u / h, kb = u - i * h;
                    int pb, qb;
                    rr_pair(m, round, kb, pb, qb);
                    if (qb >= n) continue;
                    const Rot Rb = rot[kb];
                    const Z vp = Vs[i * n + pb], vq = Vs[i * n + qb];
                    const Z j10b = zscale(Rb.e, -Rb.s), j11b = zscale(Rb.e, Rb.c);
                    Vs[i * n + pb] = zadd(zscale(vp, Rb.c), zmul(vq, j10b));
                    Vs[i * n + qb] = zadd(zscale(vp, Rb.s), zmul(vq, j11b));
                }
            }
            __syncthreads();
        }
        double off = 0.0, tot = 0.0;
        for (int e = t; e < n * n; e += nt) {
            const Z v = As[e];
            const double mm = v.x * v.x + v.y * v.y;
            tot += mm;
            if (e / n != e % n) off += mm;
        }
        red[0][t] = off;
        red[1][t] = tot;
        __syncthreads();
        for (int st = nt / 2; st > 0; st >>= 1) {
            if (t < st) {
                red[0][t] += red[0][t + st];
                red[1][t] += red[1][t + st];
            }
            __syncthreads();
        }
        const double o = sqrt(red[0][0]), tt = sqrt(red[1][0]);
        __syncthreads();   // red is reused by the next sweep
        if (!isfinite(o)) {
            result = -2;
            break;
        }
        if (o <= 1e-15 * tt || (o <= 1e-12 * tt && o >= 0.5 * prev)) {
            result = sweep + 1;
            break;
        }
        prev = o;
    }
    if (n == 1) result = 0;
    for (int j = t; j < n; j += nt) {
        const double dj = As[j * n + j].x;
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double di = As[i * n + i].x;
            rank += (di < dj) || (di == dj && i < j);
        }
        w[rank] = dj;
        for (int i = 0; i < n; ++i) Y[(int64_t)i * n + rank] = Vs[i * n + j];
    }
    if (t == 0) *status = result;
}

__global__ __launch_bounds__(1024) void k_jacobi_small(const Z *__restrict__ A0, int n,
                                                       int max_sweeps, double *__restrict__ w,
                                                       Z *__restrict__ Y, int *status) {
    __shared__ Z As[kJacobiLds * kJacobiLds];
    __shared__ Z Vs[kJacobiLds * kJacobiLds];
    __shared__ Rot rot[kJacobiLds / 2];
    __shared__ double red[2][1024];
    jacobi_all_sweeps(A0, As, Vs, rot, red, n, max_sweeps, w, Y, status);
}

// off^2 = sum_{i != j} |A_ij|^2 and tot^2 = sum |A_ij|^2 (one workgroup,
// fixed order) into out[0..1]; out[2..3] get what out[0..1] held.
__global__ __launch_bounds__(1024) void k_offnorm(const Z *__restrict__ A,
                                                  int n, double *out) {
    __shared__ double s1[1024], s2[1024];
    const int t = threadIdx.x;
    double off = 0.0, tot = 0.0;
    for (int64_t e = t; e < (int64_t)n * n; e += 1024) {
        const Z v = A[e];
        const double m = v.x * v.x + v.y * v.y;
        tot += m;
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (i != j) off += m;
    }
    s1[t] = off;
    s2[t] = tot;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (t < s) {
            s1[t] += s1[t + s];
            s2[t] += s2[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        // The previous sweep's norms move to out[2..3], so a batch of sweeps
        // checked at once still has the last two.
        const double o0 = out[0], o1 = out[1];
        out[2] = o0;
        out[3] = o1;
        out[0] = s1[0];
        out[1] = s2[0];
    }
}

__global__ void k_identity(Z *V, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e - i * n;
        V[e] = Z{i == j ? 1.0 : 0.0, 0.0};
    }
}

// Ascending order of the diagonal (ties keep index order): w[rank] and
// Y[:, rank] = V[:, j].
__global__ void k_sort_eig(const Z *__restrict__ A, const Z *__restrict__ V,
                           int n, double *w, Z *Y) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += gridDim.x * blockDim.x) {
        const double dj = A[(int64_t)j * n + j].x;
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double di = A[(int64_t)i * n + i].x;
            rank += (di < dj) || (di == dj && i < j);
        }
        w[rank] = dj;
        for (int i = 0; i < n; ++i) Y[(int64_t)i * n + rank] = V[(int64_t)i * n + j];
    }
}

__global__ void k_hermitise(Z *G, int n) {
    const int64_t total = (int64_t)n * n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
        if (j < i) continue;
        if (i == j) {
            G[e].y = 0.0;
            continue;
        }
        const Z a = G[e], b = G[(int64_t)j * n + i];
        const Z m{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
        G[e] = m;
        G[(int64_t)j * n + i] = Z{m.x, -m.y};
    }
}

inline int grid_for(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
}

}  // namespace

size_t chol_work_elems(int n) {
    const size_t np = chol_np(n), nt = np / 16;
    return 2 * np * np + nt * 256 + (np + 1) / 2 + 1;
}

void chol_qr_factor(const Z *G, int n, double shift, Z *B, Z *work, int *info,
                    hipStream_t s) {
    if (n < 1 || n > 1024) throw Error(7, "chol_qr_factor: order out of range");
    hipLaunchKernelGGL(k_chol_blocked, dim3(1), dim3(kCholThreads), 0, s, G, n, shift, B, work,
                       info);
    check_launch("k_chol_blocked");
}

size_t jacobi_work_elems(int n) { return (size_t)3 * n * n; }

void hermitise(Z *G, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_hermitise, dim3(grid_for((int64_t)n * n)), dim3(256),
                       0, s, G, n);
    check_launch("k_hermitise");
}

// A (overwritten) -> w ascending, Y eigenvectors.  work: 3 n^2 complex.
// hwork: 2 doubles of pinned host memory for the convergence test.
JacobiGraphs::~JacobiGraphs() {
    // A replay may still be queued (an error unwound the solve).
    if (!entries.empty()) (void)hipStreamSynchronize(used);
    for (auto &e : entries)
        for (auto x : e.exec)
            if (x) (void)hipGraphExecDestroy(x);
}

namespace {

// One sweep: m - 1 rounds ping-ponging (A, V) <-> (A2, V2), then the
// off-diagonal norm of the result.
void launch_sweep(Z *A, Z *A2, Z *V, Z *V2, int n, int m, int grid, double *dnorm,
                  hipStream_t s) {
    for (int r = 0; r < m - 1; ++r) {
        hipLaunchKernelGGL(k_jacobi_round, dim3(grid), dim3(256), 0, s, A, A2, V, V2, n, m, r);
        std::swap(A, A2);
        std::swap(V, V2);
    }
    check_launch("k_jacobi_round");
    hipLaunchKernelGGL(k_offnorm, dim3(1), dim3(1024), 0, s, A, n, dnorm);
    check_launch("k_offnorm");
}

// Appends one kernel node after `dep` (none if null); returns the node.
template <typename... Args>
hipGraphNode_t add_kernel(hipGraph_t g, hipGraphNode_t dep, void (*fn)(Args...), dim3 grid,
                          dim3 block, Args... args) {
    void *argp[] = {static_cast<void *>(&args)...};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = argp;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    CHASE_HIP(hipGraphAddKernelNode(&node, g, dep ? &dep : nullptr, dep ? 1 : 0, &kp));
    return node;
}

// The two sweep graphs for this order and these buffers (parity 0 starts
// from (A, V), parity 1 from (A2, V2)), built node by node on first use:
// a chain of the m - 1 round kernels and the off-norm kernel.  Building the
// graph explicitly (no stream capture) leaves every stream of the process
// free to work meanwhile.
const hipGraphExec_t *sweep_graphs(JacobiGraphs &g, Z *A, Z *A2, Z *V, Z *V2, int n, int m,
                                   int grid, double *dnorm, Z *work) {
    for (auto &e : g.entries)
        if (e.n == n && e.A == A && e.work == work) return e.exec;
    JacobiGraphs::Entry e{n, A, work, {nullptr, nullptr}, 0};
    for (int par = 0; par < 2; ++par) {
        hipGraph_t gr = nullptr;
        CHASE_HIP(hipGraphCreate(&gr, 0));
        hipError_t ie = hipSuccess;
        try {
            Z *a = par ? A2 : A, *a2 = par ? A : A2;
            Z *v = par ? V2 : V, *v2 = par ? V : V2;
            hipGraphNode_t last = nullptr;
            for (int r = 0; r < m - 1; ++r) {
                last = add_kernel(gr, last, k_jacobi_round, dim3(grid), dim3(256),
                                  static_cast<const Z *>(a), a2, static_cast<const Z *>(v),
                                  v2, n, m, r);
                std::swap(a, a2);
                std::swap(v, v2);
            }
            add_kernel(gr, last, k_offnorm, dim3(1), dim3(1024), static_cast<const Z *>(a), n,
                       dnorm);
            ie = hipGraphInstantiate(&e.exec[par], gr, nullptr, nullptr, 0);
        } catch (...) {
            (void)hipGraphDestroy(gr);
            for (auto x : e.exec)
                if (x) (void)hipGraphExecDestroy(x);
            throw;
        }
        (void)hipGraphDestroy(gr);
        if (ie != hipSuccess) {
            for (auto x : e.exec)
                if (x) (void)hipGraphExecDestroy(x);
            throw Error(3, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
    }
    g.entries.push_back(e);
    return g.entries.back().exec;
}

}  // namespace

// Sweeps the last problem of this order and buffer set needed (0 before the
// first); the entry exists once sweep_graphs has built it.
static int *graphs_last_sweeps(JacobiGraphs &g, const Z *A, int n, const Z *work) {
    for (auto &e : g.entries)
        if (e.n == n && e.A == A && e.work == work) return &e.last_sweeps;
    return nullptr;
}

static int jacobi_max_sweeps() {
    // Cyclic Jacobi converges quadratically (a few sweeps to the rounding
    // floor at these orders); a diagnostic override of the cap lets the
    // failure path be exercised.
    int max_sweeps = 30;
    if (const char *e = std::getenv("CHASE_JACOBI_MAX_SWEEPS")) {
        const int v = std::atoi(e);
        if (v >= 1) max_sweeps = v;
    }
    return max_sweeps;
}

void jacobi_check_status(int n, int st) {
    if (n > kJacobiLds) return;   // the sweep path checks as it goes
    if (st == -2) throw Error(5, "jacobi: non-finite matrix");
    if (st == -1)
        throw Error(7, "jacobi: the reduced eigenproblem did not converge in " +
                           std::to_string(jacobi_max_sweeps()) + " sweeps");
}

void jacobi_eig(Z *A, int n, double *w, Z *Y, Z *work, double *hwork,
                hipStream_t s, JacobiGraphs *graphs, int *hstatus) {
    if (n <= kJacobiLds) {
        // One launch, no host round trip per sweep; the status word lives
        // in the (otherwise unused) work buffer.  At most 8 waves, so that
        // the launch fits beside other kernels.
        const int max_sweeps = jacobi_max_sweeps();
        int *dstatus = reinterpret_cast<int *>(work);
        const int threads = n <= 32 ? 256 : 512;
        hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(threads), 0, s, (const Z *)A, n,
                           max_sweeps, w, Y, dstatus);
        check_launch("k_jacobi_small");
        if (hstatus) {
            CHASE_HIP(hipMemcpyAsync(hstatus, dstatus, sizeof(int), hipMemcpyDeviceToHost, s));
            return;
        }
        CHASE_HIP(hipMemcpyAsync(hwork, dstatus, sizeof(int), hipMemcpyDeviceToHost, s));
        CHASE_HIP(hipStreamSynchronize(s));
        int st = 0;
        std::memcpy(&st, hwork, sizeof(int));
        jacobi_check_status(n, st);
        return;
    }
    Z *A2 = work;
    Z *V = work + (size_t)n * n;
    Z *V2 = work + (size_t)2 * n * n;
    hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)n * n)), dim3(256), 0,
                       s, V, n);
    check_launch("k_identity");
    if (n > 1) {
        const int m = n + (n & 1);
        const int h = m / 2;
        const int grid = grid_for((int64_t)h * h + (int64_t)n * h);
        double *dnorm = reinterpret_cast<double *>(Y);   // Y is free until the end
        const hipGraphExec_t *ex =
            graphs ? sweep_graphs(*graphs, A, A2, V, V2, n, m, grid, dnorm, work) : nullptr;
        double prev = 1e300;
        const int max_sweeps = jacobi_max_sweeps();
        bool converged = false;
        // With sweep graphs, the first check comes after one sweep fewer
        // than the previous problem of this order needed (the reduced
        // problems of consecutive iterations are alike), then after every
        // sweep: fewer host round trips, a sweep more at most.
        int *last = graphs ? graphs_last_sweeps(*graphs, A, n, work) : nullptr;
        int batch = last ? std::max(1, *last - 1) : 1;
        int sweep = 0;
        while (sweep < max_sweeps) {
            const int b = std::min(batch, max_sweeps - sweep);
            for (int i = 0; i < b; ++i, ++sweep) {
                // m - 1 (odd) rounds: each sweep leaves the result in the
                // other buffer of the pair, so consecutive sweeps alternate
                // parity.
                if (ex) {
                    graphs->used = s;
                    CHASE_HIP(hipGraphLaunch(ex[sweep & 1], s));
                }
                else launch_sweep(A, A2, V, V2, n, m, grid, dnorm, s);
                std::swap(A, A2);
                std::swap(V, V2);
            }
            CHASE_HIP(hipMemcpyAsync(hwork, dnorm, 4 * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
            CHASE_HIP(hipStreamSynchronize(s));
            const double off = std::sqrt(hwork[0]), tot = std::sqrt(hwork[1]);
            if (b >= 2) prev = std::sqrt(hwork[2]);   // the sweep before the last
            if (!std::isfinite(off)) throw Error(5, "jacobi: non-finite matrix");
            if (off <= 1e-15 * tot || (off <= 1e-12 * tot && off >= 0.5 * prev)) {
                converged = true;   // tiny, or at the rounding floor
                break;
            }
            prev = off;
            batch = 1;
        }
        if (last) *last = sweep;
        if (!converged)
            throw Error(7, "jacobi: the reduced eigenproblem did not converge in " +
                               std::to_string(max_sweeps) + " sweeps");
    }
    hipLaunchKernelGGL(k_sort_eig, dim3((n + 255) / 256), dim3(256), 0, s, A, V,
                       n, w, Y);
    check_launch("k_sort_eig");
}


// ------------------------------------------------ allocation-free Jacobi
// Scratch of jacobi_eig_noalloc: the working copy of G, the three Jacobi
// buffers and the eigenvalues of one reduced problem of order up to
// kNoAllocMaxOrder (4 n^2 complex + n doubles = 16 MiB + 4 KiB at 512).
// Each GPU holds its own copy for the life of the process.  Host code
// never names the array itself (in host code its name is a host-side
// stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns on each device.
constexpr size_t kNoAllocScratchBytes = ((size_t)16 << 20) + ((size_t)64 << 10);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static_assert((size_t)4 * kNoAllocMaxOrder * kNoAllocMaxOrder * sizeof(Z) +
                      (size_t)kNoAllocMaxOrder * sizeof(double) + 256 <=
                  kNoAllocScratchBytes,
              "scratch too small for the largest order");

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu[kNoAllocDevices];    // one solve at a time per GPU
void *g_noalloc_ptr[kNoAllocDevices] = {};   // device address of scratch

}  // namespace

void jacobi_eig_noalloc(const Z *G, int n, double *h_w, Z *Y, hipStream_t s) {
    if (n < 1 || n > kNoAllocMaxOrder)
        throw Error(1, "order " + std::to_string(n) + " exceeds the allocation-free limit of " +
                           std::to_string(kNoAllocMaxOrder));
    int dev = -1;
    CHASE_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) throw Error(1, "device index out of range");
    // Calls are synchronous, so holding the device's lock for the call keeps
    // concurrent calls on one GPU from sharing the array at the same time.
    std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        CHASE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(3, "hipGetSymbolAddress returned NULL for the scratch array");
        g_noalloc_ptr[dev] = p;
    }
    char *base = static_cast<char *>(g_noalloc_ptr[dev]);
    const size_t nn = (size_t)n * n;
    Z *A = reinterpret_cast<Z *>(base);
    Z *work = A + nn;                                          // 3 n^2
    double *w = reinterpret_cast<double *>(work + jacobi_work_elems(n));
    double hw[4];
    CHASE_HIP(hipMemcpyAsync(A, G, nn * sizeof(Z), hipMemcpyDeviceToDevice, s));
    jacobi_eig(A, n, w, Y, work, hw, s, nullptr);
    CHASE_HIP(hipMemcpyAsync(h_w, w, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    CHASE_HIP(hipStreamSynchronize(s));
}

}  // namespace chase
