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
// CholeskyQR factor, one workgroup of 1024 threads: G (n x n row-major,
// n <= 1024) -> B = D L^{-H} (upper triangular, row-major) with L the lower
// Cholesky factor of D G D + shift I and D = diag(G)^{-1/2}.  `work` holds
// D and X = L^{-1}.  *info = 0, or k + 1 for a non-positive pivot k (then
// B is not written).  Both halves are right-looking, one step per column:
//  * Cholesky step k: scale column k by 1/sqrt(pivot), then subtract the
//    rank-1 product of column k from the trailing lower triangle;
//  * inversion step k: X[k][j] *= 1/L[k][k] for j <= k, then
//    X[i][j] -= L[i][k] X[k][j] for i > k, j <= k.
// Each step's serial input (column k of the updated matrix, with its
// pivot; row k of X) is handed over through LDS by the previous step's
// update instead of being re-read from memory, so a step waits on L2 once
// (its own update) rather than three times.

__global__ __launch_bounds__(1024) void k_chol_factor(Z *G, int n, double shift,
                                                      Z *B, Z *work,
                                                      int *info) {
    __shared__ int bad;
    __shared__ Z colk[1024], nxt[1024], rowk[1024];
    __shared__ double ldiag[1024];
    const int t = threadIdx.x, nt = blockDim.x;
    double *dsc = reinterpret_cast<double *>(work);          // n doubles
    Z *X = work + (n + 1) / 2 + 1;                           // n x n
    if (t == 0) bad = 0x7fffffff;
    __syncthreads();
    for (int j = t; j < n; j += nt) {
        const double gjj = G[(int64_t)j * n + j].x;
        if (!(gjj > 0.0) || !isfinite(gjj)) atomicMin(&bad, j + 1);   // LDS atomic
        dsc[j] = gjj > 0.0 ? 1.0 / sqrt(gjj) : 0.0;
    }
    __syncthreads();
    if (bad != 0x7fffffff) {
        if (t == 0) *info = bad;
        return;
    }
    // Scale and shift (lower triangle only is used below); X = I; column 0
    // of the scaled matrix into LDS.
    for (int e = t; e < n * n; e += nt) {
        const int i = e / n, j = e - i * n;
        X[e] = Z{i == j ? 1.0 : 0.0, 0.0};
        if (j > i) continue;
        Z v = zscale(G[e], dsc[i] * dsc[j]);
        if (i == j) v = Z{v.x + shift, 0.0};
        G[e] = v;
        if (j == 0) nxt[i] = v;
    }
    __syncthreads();
    // Right-looking Cholesky, lower.  nxt holds column k (rows >= k).
    for (int k = 0; k < n; ++k) {
        const double piv = nxt[k].x;
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (t == 0) *info = k + 1;
            return;   // uniform: every thread read the same pivot
        }
        const double l = sqrt(piv), il = 1.0 / l;
        for (int i = k + 1 + t; i < n; i += nt) {
            const Z v = zscale(nxt[i], il);
            G[(int64_t)i * n + k] = v;
            colk[i] = v;
        }
        if (t == 0) {
            G[(int64_t)k * n + k] = Z{l, 0.0};
            ldiag[k] = l;
        }
        __syncthreads();
        const int m = n - k - 1;
        for (int e = t; e < m * m; e += nt) {
            const int ii = e / m, jj = e - ii * m;
            if (jj > ii) continue;
            const int i = k + 1 + ii, j = k + 1 + jj;
            const Z v = zsub(G[(int64_t)i * n + j], zmul(colk[i], zconj(colk[j])));
            G[(int64_t)i * n + j] = v;
            if (jj == 0) nxt[i] = v;   // column k + 1 for the next step
        }
        __syncthreads();
    }
    // X = L^{-1}, right-looking.  rowk holds row k of X (entries <= k);
    // thread t prefetches L[k + 2 + t][k + 1] for the next step.
    if (t == 0) nxt[0] = Z{1.0, 0.0};
    Z lnext = (1 + t < n) ? G[(int64_t)(1 + t) * n + 0] : Z{0.0, 0.0};
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double xkk = 1.0 / ldiag[k];
        for (int j = t; j <= k; j += nt) {
            const Z x = zscale(nxt[j], xkk);
            X[(int64_t)k * n + j] = x;
            rowk[j] = x;
        }
        if (k + 1 + t < n) colk[k + 1 + t] = lnext;
        if (k + 2 + t < n) lnext = G[(int64_t)(k + 2 + t) * n + (k + 1)];
        __syncthreads();
        const int w = k + 1, m = n - k - 1;
        for (int e = t; e < m * w; e += nt) {
            const int ii = e / w, j = e - ii * w;
            const int i = k + 1 + ii;
            const Z v = zsub(X[(int64_t)i * n + j], zmul(colk[i], rowk[j]));
            X[(int64_t)i * n + j] = v;
            if (ii == 0) nxt[j] = v;   // row k + 1 for the next step
        }
        if (t == 0 && k + 1 < n) nxt[k + 1] = Z{1.0, 0.0};
        __syncthreads();
    }
    for (int e = t; e < n * n; e += nt) {
        const int j = e / n, i = e - j * n;   // B row j, column i
        B[e] = i >= j ? zscale(zconj(X[(int64_t)i * n + j]), dsc[j]) : Z{0.0, 0.0};
    }
    if (t == 0) *info = 0;
}

// The same factor with the matrix held in LDS for orders up to
// kCholLds: the packed lower triangle (entry (i, j), j <= i, at
// i (i + 1) / 2 + j; 158 KB at n = 140), one column and the scale factors
// fit gfx950's 160 KB, so no step waits on L2.  Same operations in the same
// order as k_chol_factor; X = L^{-1} overwrites L in place (column k of L is
// saved before row k of X takes its place), and the (row, column) loops run
// on a 32 x 32 thread grid instead of dividing a flat index.
constexpr int kCholLds = 140;

__global__ __launch_bounds__(1024) void k_chol_factor_lds(const Z *G, int n, double shift,
                                                          Z *B, int *info) {
    __shared__ Z T[kCholLds * (kCholLds + 1) / 2];
    __shared__ Z colk[kCholLds];
    __shared__ double dsc[kCholLds];
    __shared__ int bad;
    const int t = threadIdx.x, nt = blockDim.x;
    const int tr = t >> 5, tc = t & 31;
    auto at = [](int i, int j) { return i * (i + 1) / 2 + j; };
    if (t == 0) bad = 0x7fffffff;
    __syncthreads();
    for (int j = t; j < n; j += nt) {
        const double gjj = G[(int64_t)j * n + j].x;
        if (!(gjj > 0.0) || !isfinite(gjj)) atomicMin(&bad, j + 1);   // LDS atomic
        dsc[j] = gjj > 0.0 ? 1.0 / sqrt(gjj) : 0.0;
    }
    __syncthreads();
    if (bad != 0x7fffffff) {
        if (t == 0) *info = bad;
        return;
    }
    for (int i = tr; i < n; i += 32)
        for (int j = tc; j <= i; j += 32) {
            Z v = zscale(G[(int64_t)i * n + j], dsc[i] * dsc[j]);
            if (i == j) v = Z{v.x + shift, 0.0};
            T[at(i, j)] = v;
        }
    __syncthreads();
    // Right-looking Cholesky, lower.
    for (int k = 0; k < n; ++k) {
        const double piv = T[at(k, k)].x;
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (t == 0) *info = k + 1;
            return;   // uniform: every thread read the same pivot
        }
        const double l = sqrt(piv), il = 1.0 / l;
        __syncthreads();   // the pivot is read everywhere before it is replaced
        for (int i = k + 1 + t; i < n; i += nt) {
            const Z v = zscale(T[at(i, k)], il);
            T[at(i, k)] = v;
            colk[i] = v;
        }
        if (t == 0) T[at(k, k)] = Z{l, 0.0};
        __syncthreads();
        for (int i = k + 1 + tr; i < n; i += 32) {
            const Z ci = colk[i];
            for (int j = k + 1 + tc; j <= i; j += 32)
                T[at(i, j)] = zsub(T[at(i, j)], zmul(ci, zconj(colk[j])));
        }
        __syncthreads();
    }
    // X = L^{-1} in place, right-looking: X[k][j] *= 1/L[k][k] (j <= k, with
    // X[k][k] = 1 before), then X[i][j] -= L[i][k] X[k][j] for i > k
    // (X[i][k] = 0 before).
    for (int k = 0; k < n; ++k) {
        for (int i = k + 1 + t; i < n; i += nt) colk[i] = T[at(i, k)];
        const double xkk = 1.0 / T[at(k, k)].x;
        __syncthreads();
        for (int j = t; j <= k; j += nt)
            T[at(k, j)] = zscale(j == k ? Z{1.0, 0.0} : T[at(k, j)], xkk);
        __syncthreads();
        for (int i = k + 1 + tr; i < n; i += 32) {
            const Z ci = colk[i];
            for (int j = tc; j <= k; j += 32) {
                const Z cur = j == k ? Z{0.0, 0.0} : T[at(i, j)];
                T[at(i, j)] = zsub(cur, zmul(ci, T[at(k, j)]));
            }
        }
        __syncthreads();
    }
    for (int j = tr; j < n; j += 32)          // B row j, column i
        for (int i = tc; i < n; i += 32)
            B[(int64_t)j * n + i] = i >= j ? zscale(zconj(T[at(i, j)]), dsc[j]) : Z{0.0, 0.0};
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

// off^2 = sum_{i != j} |A_ij|^2 and tot^2 = sum |A_ij|^2 (one workgroup,
// fixed order).
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

void chol_qr_factor(Z *G, int n, double shift, Z *B, Z *work, int *info,
                    hipStream_t s) {
    if (n <= kCholLds) {
        hipLaunchKernelGGL(k_chol_factor_lds, dim3(1), dim3(1024), 0, s, (const Z *)G, n, shift,
                           B, info);
        check_launch("k_chol_factor_lds");
        return;
    }
    hipLaunchKernelGGL(k_chol_factor, dim3(1), dim3(1024), 0, s, G, n, shift, B, work,
                       info);
    check_launch("k_chol_factor");
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
    JacobiGraphs::Entry e{n, A, work, {nullptr, nullptr}};
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

void jacobi_eig(Z *A, int n, double *w, Z *Y, Z *work, double *hwork,
                hipStream_t s, JacobiGraphs *graphs) {
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
        // Cyclic Jacobi converges quadratically (a few sweeps to the rounding
        // floor at these orders); a diagnostic override of the cap lets the
        // failure path be exercised.
        int max_sweeps = 30;
        if (const char *e = std::getenv("CHASE_JACOBI_MAX_SWEEPS")) {
            const int v = std::atoi(e);
            if (v >= 1) max_sweeps = v;
        }
        bool converged = false;
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
            // m - 1 (odd) rounds: each sweep leaves the result in the other
            // buffer of the pair, so consecutive sweeps alternate parity.
            if (ex) {
                graphs->used = s;
                CHASE_HIP(hipGraphLaunch(ex[sweep & 1], s));
            }
            else launch_sweep(A, A2, V, V2, n, m, grid, dnorm, s);
            std::swap(A, A2);
            std::swap(V, V2);
            CHASE_HIP(hipMemcpyAsync(hwork, dnorm, 2 * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
            CHASE_HIP(hipStreamSynchronize(s));
            const double off = std::sqrt(hwork[0]), tot = std::sqrt(hwork[1]);
            if (!std::isfinite(off)) throw Error(5, "jacobi: non-finite matrix");
            if (off <= 1e-15 * tot || (off <= 1e-12 * tot && off >= 0.5 * prev)) {
                converged = true;   // tiny, or at the rounding floor
                break;
            }
            prev = off;
        }
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
