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
#include <type_traits>
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
// CholeskyQR factor, two launches: k_chol_prep writes W = D G D + shift I
// (one workgroup per 16 x 16 tile), then one workgroup of 8 waves factors
// it: G (n x n Hermitian, row-major, n <= 1024, not modified) -> B =
// D L^{-H} (upper triangular, row-major) with L the lower Cholesky factor
// of W and D = diag(G)^{-1/2}, so that V <- V B orthonormalises.  *info = 0, or
// j + 1 for the first non-positive (or non-finite) pivot j (then B is not
// complete).
//
// Blocked in 16 x 16 complex blocks (nt = ceil(n / 16) per side; W is
// padded with the identity to 16 nt, which leaves L and L^{-1} padded with
// the identity), right-looking with a look-ahead of one diagonal block.
// Step k, after the inverse of the diagonal block L_kk is known:
//  * phase P: the panel L_ik = W_ik L_kk^{-H} (i > k), staged in LDS as
//    well, and X_kk = L_kk^{-1} (X = L^{-1});
//  * phase T: wave 0 updates W_{k+1,k+1} and factors and inverts it
//    (diag_factor) while the other waves do block row k of X,
//    X_kj = -L_kk^{-1} sum_{m=j}^{k-1} L_km X_mj (j < k, whose operands were
//    final at earlier steps), and the rest of the trailing update
//    W_ij -= L_ik L_jk^H (k < j <= i).
// Block products are 16 x 16 x 16 complex on FP64 MFMA.  Every X block is
// written to B (conjugate transpose, scaled) by the wave that forms it.
// Two workgroup barriers per step.  W, X and D live in `work`
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

// 8 waves (2 per SIMD): room is left on the CU for other kernels.
constexpr int kCholThreads = 512;
constexpr int kCholWaves = kCholThreads / 64;
// Panel blocks staged in LDS (n <= 16 (kPanelLds + 1)); beyond, the
// trailing update reads them from W.
constexpr int kPanelLds = 32;

size_t chol_np(int n) { return (size_t)(n + 15) / 16 * 16; }

// Orders the LDS accesses of one wave's lanes (no other wave is involved).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Calls f(integral_constant<int, I>) for I = B .. E-1 (compile-time indices,
// as the DPP lane selects below need).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// The double held by lane M of each row of 16 lanes, to every lane of that
// row (DPP row_newbcast).
template <int M>
__device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + M, 0xf, 0xf, false);   // one 64-bit DPP move
}

// One wave: the 16 x 16 diagonal block in Ls (lower part; the wave's own
// writes, ordered before the call) -> L^{-1} (its Cholesky factor's
// inverse) in linv.  Lane i (of every row of
// 16 lanes: the four rows hold the same data) keeps row i in registers;
// column j's pivot and entries reach the other lanes by DPP broadcasts, so
// no LDS round trip per column and no workgroup barrier falls inside.  Then
// L goes to Ls and lane c forms column c of L^{-1} by forward substitution.
// Returns j + 1 for a non-positive or non-finite pivot j (linv then
// unwritten), else 0.
__device__ __forceinline__ int diag_factor(Z (*Ls)[17], Z (*linv)[17]) {
    const int lane = threadIdx.x & 63, i = lane & 15;
    Z a[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) a[m] = m <= i ? Ls[i][m] : Z{0.0, 0.0};
    double il[16];
    int bad = 0;
    static_for<0, 16>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (bad) return;
        const double piv = row_bcast<j>(a[j].x);   // the same in every lane
        if (!(piv > 0.0) || !isfinite(piv)) {
            bad = j + 1;
            return;
        }
        const double rl = rsqrt(piv);
        il[j] = rl;
        if (i > j) a[j] = zscale(a[j], rl);
        else if (i == j) a[j] = Z{piv * rl, 0.0};
        // a[i][m] -= L_ij conj(L_mj), m > j (entries above the diagonal are
        // updated too and never read).
        static_for<j + 1, 16>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const Z lm{row_bcast<m>(a[j].x), row_bcast<m>(a[j].y)};
            // a[m] -= a[j] conj(lm), four fused multiply-adds
            a[m].x = fma(-a[j].x, lm.x, fma(-a[j].y, lm.y, a[m].x));
            a[m].y = fma(a[j].x, lm.y, fma(-a[j].y, lm.x, a[m].y));
        });
    });
    if (bad) return bad;
    // L to LDS by rows, then column c of L^{-1}, x_r = (delta_rc -
    // sum_{m<r} L_rm x_m) / L_rr, right-looking (x_r is final at step r and
    // is then subtracted from the rows below it at once, which keeps the
    // dependent chain at 16 steps; each x_r's terms are still added in the
    // order m = 0, 1, ...), reading L back as broadcasts.
    if (lane < 16) {
#pragma unroll
        for (int m = 0; m < 16; ++m) Ls[i][m] = a[m];
    }
    wave_sync();
    Z x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = Z{i == r ? 1.0 : 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        x[j] = zscale(x[j], il[j]);
#pragma unroll
        for (int r = j + 1; r < 16; ++r) {
            const Z l = Ls[r][j];   // x[r] -= l x[j]
            x[r].x = fma(l.y, x[j].y, fma(-l.x, x[j].x, x[r].x));
            x[r].y = fma(-l.y, x[j].x, fma(-l.x, x[j].y, x[r].y));
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) linv[r][i] = x[r];
    }
    return 0;
}

// W = D G D + shift I (D = diag(G)^(-1/2)) in its lower triangle, padded
// with the identity to 16 nt, and B's blocks below the diagonal blocks set
// to zero: one 16 x 16 tile per workgroup over the lower tiles (tile b =
// (I, J), row-major over J <= I), so this O(n^2) pass is spread over the
// chip rather than left to the factor's single workgroup.
__global__ __launch_bounds__(256) void k_chol_prep(const Z *__restrict__ G, int n, double shift,
                                                   Z *__restrict__ B, Z *__restrict__ W) {
    const int np = 16 * ((n + 15) / 16);
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (I > 0 && I * (I + 1) / 2 > b) --I;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    const int J = b - I * (I + 1) / 2;
    const int i = 16 * I + (int)(threadIdx.x >> 4), j = 16 * J + (int)(threadIdx.x & 15);
    if (j <= i) {
        Z v{i == j ? 1.0 : 0.0, 0.0};
        if (i < n) {
            const double gi = G[(int64_t)i * n + i].x, gj = G[(int64_t)j * n + j].x;
            const double di = gi > 0.0 ? 1.0 / sqrt(gi) : 0.0;
            const double dj = gj > 0.0 ? 1.0 / sqrt(gj) : 0.0;
            v = zscale(G[(int64_t)i * n + j], di * dj);
            if (i == j) v = Z{v.x + shift, 0.0};
        }
        W[(int64_t)i * np + j] = v;
    }
    if (I > J && i < n && j < n) B[(int64_t)i * n + j] = Z{0.0, 0.0};
}

__global__ __launch_bounds__(kCholThreads) void k_chol_blocked(const Z *__restrict__ G, int n,
                                                               Z *__restrict__ B,
                                                               Z *__restrict__ work,
                                                               int *info) {
    __shared__ Z linv[2][16][17];          // L_kk^{-1}, by step parity
    __shared__ Z Lp[kPanelLds][16][17];    // the panel L_ik, i = k + 1 + index
    __shared__ Z Ls[16][17];               // the diagonal block's factor
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int nt = (n + 15) / 16, np = 16 * nt;
    const bool lds_panel = nt - 1 <= kPanelLds;
    Z *W = work;                                  // np x np, row-major
    Z *X = W + (size_t)np * np;                   // np x np: L^{-1}
    double *dsc = reinterpret_cast<double *>(X + (size_t)np * np);   // np

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
    // W (the scaled, shifted, padded lower triangle) and the zero blocks of
    // B were written by k_chol_prep.

    // Block (i, k) of X, in accumulator layout, to X and to B = D X^H.
    auto put_x = [&](int i, int k, const v4d &xr, const v4d &xi) {
        Z *Xik = X + (int64_t)16 * i * np + 16 * k;
        const int brow = 16 * k + r;
        const double sc = brow < n ? dsc[brow] : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Xik[(int64_t)(q + 4 * v) * np + r] = Z{xr[v], xi[v]};
            const int bcol = 16 * i + q + 4 * v;
            if (brow < n && bcol < n)
                B[(int64_t)brow * n + bcol] = Z{xr[v] * sc, -xi[v] * sc};
        }
    };

    if (wave == 0) {
        for (int e = lane; e < 256; e += 64) Ls[e >> 4][e & 15] = W[(e >> 4) * np + (e & 15)];
        wave_sync();
        const int b0 = diag_factor(Ls, linv[0]);
        if (b0 && lane == 0) bad = b0;
    }
    __syncthreads();
    if (bad != 0x7fffffff) {
        if (t == 0) *info = bad;
        return;
    }

    for (int k = 0; k < nt; ++k) {
        const int64_t kk0 = (int64_t)16 * k;
        Z (*li)[17] = linv[k & 1];
        // ---- phase P: X_kk and the panel L_ik = W_ik L_kk^{-H}, i > k.
        // Wave 0 also fetches W_{k+1,k+1} (final since the last step) for
        // its update in phase T.
        v4d dr{0, 0, 0, 0}, di{0, 0, 0, 0};
        if (wave == 0 && k + 1 < nt) {
            const Z *Wii = W + (int64_t)16 * (k + 1) * np + 16 * (k + 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Z w = Wii[(int64_t)(q + 4 * v) * np + r];
                dr[v] = w.x;
                di[v] = w.y;
            }
        }
        if (wave == 0) {
            v4d xr, xi;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                xr[v] = li[q + 4 * v][r].x;
                xi[v] = li[q + 4 * v][r].y;
            }
            put_x(k, k, xr, xi);
        }
        for (int i = k + 1 + wave; i < nt; i += kCholWaves) {
            const Z *Wi = W + (int64_t)16 * i * np + kk0;
            v4d cr{0, 0, 0, 0}, ci{0, 0, 0, 0};
            zblock_mac(cr, ci, [&](int s) { return Wi[(int64_t)r * np + 4 * s + q]; },
                       [&](int s) { return zconj(li[r][4 * s + q]); });
            Z *Wo = W + (int64_t)16 * i * np + kk0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const Z o{cr[v], ci[v]};
                Wo[(int64_t)(q + 4 * v) * np + r] = o;
                if (lds_panel) Lp[i - k - 1][q + 4 * v][r] = o;
            }
        }
        __syncthreads();
        // ---- phase T
        if (wave == 0) {
            if (k + 1 < nt) {
                // W_{k+1,k+1} -= L_{k+1,k} L_{k+1,k}^H (the panel block from
                // LDS when staged), into Ls, then its factor.  W_{k+1,k+1}
                // itself is not read again.
                const int i = k + 1;
                if (lds_panel) {
                    zblock_mac(dr, di,
                               [&](int s) {
                                   const Z a = Lp[0][r][4 * s + q];
                                   return Z{-a.x, -a.y};
                               },
                               [&](int s) { return zconj(Lp[0][r][4 * s + q]); });
                } else {
                    const Z *Lik = W + (int64_t)16 * i * np + kk0;
                    zblock_mac(dr, di,
                               [&](int s) {
                                   const Z a = Lik[(int64_t)r * np + 4 * s + q];
                                   return Z{-a.x, -a.y};
                               },
                               [&](int s) { return zconj(Lik[(int64_t)r * np + 4 * s + q]); });
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) Ls[q + 4 * v][r] = Z{dr[v], di[v]};
                wave_sync();
                const int bi = diag_factor(Ls, linv[(k + 1) & 1]);
                if (bi && lane == 0) bad = 16 * (k + 1) + bi;
            }
        } else {
            // Jobs: X row k (j = 0 .. k-1, the longest sums first), then the
            // trailing tiles other than (k+1, k+1); round-robin over waves
            // 1 .. kCholWaves - 1.
            const int m = nt - k - 1;
            const int tiles = m * (m + 1) / 2;
            const int jobs = k + tiles;
            int u = wave - 1;
            for (; u < k; u += kCholWaves - 1) {
                {
                    const int j = u;
                    v4d cr{0, 0, 0, 0}, ci{0, 0, 0, 0};
                    const Z *Lk = W + kk0 * np;
                    Z la[4], xa[4];
                    auto load = [&](int mm, Z *lo, Z *xo) {
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            lo[s] = Lk[(int64_t)r * np + 16 * mm + 4 * s + q];
                            xo[s] = X[(int64_t)(16 * mm + 4 * s + q) * np + 16 * j + r];
                        }
                    };
                    load(j, la, xa);
                    for (int mm = j; mm < k; ++mm) {
                        Z lb[4], xb[4];
                        load(min(mm + 1, k - 1), lb, xb);   // next operands in flight
                        zblock_mac(cr, ci, [&](int s) { return la[s]; },
                                   [&](int s) { return xa[s]; });
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            la[s] = lb[s];
                            xa[s] = xb[s];
                        }
                    }
                    v4d xr{0, 0, 0, 0}, xi{0, 0, 0, 0};
                    zblock_mac(xr, xi,
                               [&](int s) {
                                   const Z a = li[r][4 * s + q];
                                   return Z{-a.x, -a.y};
                               },
                               [&](int s) { return Z{cr[s], ci[s]}; });
                    put_x(k, j, xr, xi);
                    continue;
                }
            }
            // Trailing tile number tt = u - k + 1 (row-major over k < j <= i),
            // skipping (k+1, k+1), which is tile 0.  The next tile's W is
            // loaded before the current tile's products, so its L2 latency
            // overlaps them.
            auto tile_at = [&](int uu, int &i, int &j) {
                const int tt = uu - k + 1;
                if (uu >= jobs || tt >= tiles) return false;
                int ii = (int)((sqrt(8.0 * tt + 1.0) - 1.0) * 0.5);
                while (ii * (ii + 1) / 2 > tt) --ii;
                while ((ii + 1) * (ii + 2) / 2 <= tt) ++ii;
                i = k + 1 + ii;
                j = k + 1 + tt - ii * (ii + 1) / 2;
                return true;
            };
            auto load_w = [&](int i, int j, v4d &cr, v4d &ci) {
                const Z *Wij = W + (int64_t)16 * i * np + 16 * j;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const Z w = Wij[(int64_t)(q + 4 * v) * np + r];
                    cr[v] = w.x;
                    ci[v] = w.y;
                }
            };
            int ni = 0, nj = 0;
            v4d nr{0, 0, 0, 0}, nim{0, 0, 0, 0};
            bool have = tile_at(u, ni, nj);
            if (have) load_w(ni, nj, nr, nim);
            while (have) {
                const int i = ni, j = nj;
                v4d cr = nr, ci = nim;
                u += kCholWaves - 1;
                have = tile_at(u, ni, nj);
                if (have) load_w(ni, nj, nr, nim);
                if (lds_panel) {
                    zblock_mac(cr, ci,
                               [&](int s) {
                                   const Z a = Lp[i - k - 1][r][4 * s + q];
                                   return Z{-a.x, -a.y};
                               },
                               [&](int s) { return zconj(Lp[j - k - 1][r][4 * s + q]); });
                } else {
                    const Z *Lik = W + (int64_t)16 * i * np + kk0;
                    const Z *Ljk = W + (int64_t)16 * j * np + kk0;
                    zblock_mac(cr, ci,
                               [&](int s) {
                                   const Z a = Lik[(int64_t)r * np + 4 * s + q];
                                   return Z{-a.x, -a.y};
                               },
                               [&](int s) { return zconj(Ljk[(int64_t)r * np + 4 * s + q]); });
                }
                Z *Wij = W + (int64_t)16 * i * np + 16 * j;
#pragma unroll
                for (int v = 0; v < 4; ++v) Wij[(int64_t)(q + 4 * v) * np + r] = Z{cr[v], ci[v]};
            }
        }
        __syncthreads();
        if (bad != 0x7fffffff) {
            if (t == 0) *info = bad;
            return;   // uniform: every thread reads the flag after the barrier
        }
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
        // (r + k) mod (m - 1) and (r - k) mod (m - 1), 0 <= r, k < m - 1.
        a = r + k;
        if (a >= m - 1) a -= m - 1;
        b = r - k;
        if (b < 0) b += m - 1;
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

// The rotation for the pivot pair (p, q) from a_pp, a_qq and a_pq: the
// phase e = conj(a_pq)/|a_pq| makes the pair real, then t = tan(theta) is
// the root of smaller modulus of t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp)
// / (2 |a_pq|), with c = 1/sqrt(1 + t^2) and s = t c (Golub & Van Loan
// Alg. 8.5.1 after the phase).  A round waits on this dependent chain, so
// 1/|a_pq| and c come from reciprocal square roots: one square root and one
// division remain (against three of each in the textbook form).  Returns
// the identity (active = false) when a_pq is zero or negligible.
__device__ __forceinline__ Rot rot_from(double app, double aqq, Z apq) {
    Rot R{1.0, 0.0, Z{1.0, 0.0}, app, aqq, false};
    const double s2 = apq.x * apq.x + apq.y * apq.y;
    const double r = rsqrt(s2);   // 1/|a_pq| (inf for 0, then x is NaN)
    const double x = s2 * r;
    if (!(x > 1e-300) || x <= 1e-18 * (fabs(app) + fabs(aqq))) return R;
    R.e = Z{apq.x * r, -apq.y * r};
    const double tau = (aqq - app) * (0.5 * r);
    double t;
    if (fabs(tau) > 1e150) t = 0.5 / tau;
    else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(fma(tau, tau, 1.0)));
    R.c = rsqrt(fma(t, t, 1.0));
    R.s = t * R.c;
    R.dp = app - t * x;
    R.dq = aqq + t * x;
    R.active = true;
    return R;
}

__device__ Rot make_rot(const Z *A, int n, int p, int q) {
    const double app = A[(int64_t)p * n + p].x;   // p < n always
    if (q >= n) return Rot{1.0, 0.0, Z{1.0, 0.0}, app, 0.0, false};   // phantom partner (n odd)
    return rot_from(app, A[(int64_t)q * n + q].x, A[(int64_t)p * n + q]);
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

// ------------------------------------------------ Jacobi, mid-size orders
// For kJacobiLds < n <= kJacobiMid the whole cyclic Jacobi of A runs in one
// workgroup with A Hermitian-packed in LDS (upper triangle, n (n + 1) / 2
// entries: 158 KB at n = 140), every sweep and its convergence test in one
// launch.  The eigenvectors are not formed there: each round's rotations
// (c, s, e) are recorded, and a second kernel applies them, in order, to
// the rows of the identity (each row of V is independent: one wave per row,
// the row in LDS), then writes Y in ascending eigenvalue order.  The
// rotations and the update formulas are those of k_jacobi_round.  A round's
// rotations sit in LDS as 32-byte (c, s, e) records; an update takes its
// pair indices from the round-robin formula and the packed row offsets by
// arithmetic, so its LDS reads are two records and four matrix entries
// (pair indices and offset tables read from LDS made every round 30%
// slower).
constexpr int kJacobiMid = 140;
constexpr int kJacobiMidThreads = 1024;
constexpr int kRotSweeps = 30;   // capacity of the rotation record, in sweeps

// Work layout (complex elements): [0, 64) the status words and the
// permutation (int), then 2 per rotation, kRotSweeps (m - 1) h of them.
constexpr size_t kMidHead = 64;
size_t jacobi_mid_elems(int n) {
    const size_t m = (size_t)(n + (n & 1)), h = m / 2;
    return kMidHead + 2 * (size_t)kRotSweeps * (m - 1) * h;
}

__device__ __forceinline__ int pk_idx(int x, int y, int n) {   // x <= y
    return x * (2 * n - x + 1) / 2 + (y - x);
}
// Entry (x, y) of the packed Hermitian matrix (no branch: the stored one
// and a conjugation); rb[x] = pk_idx(x, x, n) - x.
__device__ __forceinline__ Z pk_get(const Z *P, const int *rb, int x, int y) {
    Z v = P[rb[min(x, y)] + max(x, y)];
    if (x > y) v.y = -v.y;
    return v;
}
__device__ __forceinline__ void pk_set(Z *P, const int *rb, int x, int y, Z v) {
    if (x > y) v.y = -v.y;
    P[rb[min(x, y)] + max(x, y)] = v;
}
// a * b and conj(a) * b
__device__ __forceinline__ Z zmul_f(Z a, Z b) {
    return Z{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ Z zcmul_f(Z a, Z b) {
    return Z{fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x)};
}
// c x + s y and c x - s y for real c, s
__device__ __forceinline__ Z zaxpby(double c, Z x, double s, Z y) {
    return Z{fma(c, x.x, s * y.x), fma(c, x.y, s * y.y)};
}

// make_rot on the packed matrix (p < q).
__device__ Rot make_rot_packed(const Z *P, int n, int p, int q) {
    const double app = P[pk_idx(p, p, n)].x;
    if (q >= n) return Rot{1.0, 0.0, Z{1.0, 0.0}, app, 0.0, false};
    return rot_from(app, P[pk_idx(q, q, n)].x, P[pk_idx(p, q, n)]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(kJacobiMidThreads) void k_jacobi_mid(const Z *__restrict__ A0,
                                                                  int n, int max_sweeps,
                                                                  double *__restrict__ w,
                                                                  Z *__restrict__ work) {
    __shared__ Z P[kJacobiMid * (kJacobiMid + 1) / 2];
    struct RotCS {
        double c, s, ex, ey;
    };
    __shared__ RotCS rcs[kJacobiMid / 2];      // the round's rotations
    __shared__ double2 rdg[kJacobiMid / 2];    // their resulting diagonal pairs
    __shared__ int ract[kJacobiMid / 2];
    __shared__ int rb[kJacobiMid];
    __shared__ double red[2][kJacobiMidThreads / 64];
    __shared__ int decide;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nw = kJacobiMidThreads / 64;
    const int m = n + (n & 1), h = m / 2;
    int *hdr = reinterpret_cast<int *>(work);   // [0] status, [1] rounds recorded
    int *perm = hdr + 16;
    Z *rec = work + kMidHead;
    for (int x = t; x < n; x += kJacobiMidThreads) rb[x] = pk_idx(x, x, n) - x;
    for (int e = t; e < n * (n + 1) / 2; e += kJacobiMidThreads) {
        // e -> (x, y), x <= y, row-major over the upper triangle
        int x = (int)((2.0 * n + 1.0 - sqrt((2.0 * n + 1.0) * (2.0 * n + 1.0) - 8.0 * e)) * 0.5);
        while (x > 0 && pk_idx(x, x, n) > e) --x;
        while (x + 1 < n && pk_idx(x + 1, x + 1, n) <= e) ++x;
        const int y = x + (e - pk_idx(x, x, n));
        P[e] = A0[(int64_t)x * n + y];
    }
    __syncthreads();
    double prev = 1e300;
    int result = -1, rounds = 0;
    // Blocks ka <= kb, enumerated folded over hf = h rounded up to even:
    // rows ka and hf - 1 - ka together hold hf + 1 of them (those with
    // kb = h, present only when h is odd, are skipped).
    const int hf = h + (h & 1);
    const int nblk = hf / 2 * (hf + 1);
    // This thread's blocks (the same every round): at most kMidBlk.
    constexpr int kMidBlk = (kJacobiMid / 2 / 2 * (kJacobiMid / 2 + 1) + kJacobiMidThreads - 1) /
                            kJacobiMidThreads;
    int bka[kMidBlk], bkb[kMidBlk];
#pragma unroll
    for (int u = 0; u < kMidBlk; ++u) {
        const int e = t + u * kJacobiMidThreads;
        bka[u] = bkb[u] = -1;
        if (e >= nblk) continue;
        const int pr = e / (hf + 1), o = e - pr * (hf + 1);
        int ka, kb;
        if (o < hf - pr) {
            ka = pr;
            kb = pr + o;
        } else {
            ka = hf - 1 - pr;
            kb = ka + (o - (hf - pr));
        }
        if (kb >= h) continue;
        bka[u] = ka;
        bkb[u] = kb;
    }
    for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
        for (int round = 0; round < m - 1; ++round, ++rounds) {
            for (int k = t; k < h; k += kJacobiMidThreads) {
                int p, q;
                rr_pair(m, round, k, p, q);
                const Rot R = make_rot_packed(P, n, p, q);
                rcs[k] = RotCS{R.c, R.s, R.e.x, R.e.y};
                rdg[k] = double2{R.dp, R.dq};
                ract[k] = R.active ? 1 : 0;
                Z *o = rec + 2 * ((int64_t)rounds * h + k);
                o[0] = Z{R.c, R.s};
                o[1] = R.e;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kMidBlk; ++u) {
                const int ka = bka[u], kb = bkb[u];
                if (ka < 0) continue;
                // Pair indices from the round-robin formula and row offsets
                // by arithmetic (no LDS reads for either).
                int pa, qa, pb, qb;
                rr_pair(m, round, ka, pa, qa);
                rr_pair(m, round, kb, pb, qb);
                const bool qa_ok = qa < n, qb_ok = qb < n;
                auto rbx = [&](int x) { return (x * (2 * n - x - 1)) >> 1; };
                if (ka == kb) {
                    const double2 d = rdg[ka];
                    P[rbx(pa) + pa] = Z{d.x, 0.0};
                    if (qa_ok) {
                        P[rbx(qa) + qa] = Z{d.y, 0.0};
                        if (ract[ka]) P[rbx(pa) + qa] = Z{0.0, 0.0};
                    }
                    continue;
                }
                const RotCS ra = rcs[ka], rbr = rcs[kb];
                const Z ea{ra.ex, ra.ey}, eb{rbr.ex, rbr.ey};
                auto get = [&](int x, int y) {
                    Z v = P[rbx(min(x, y)) + max(x, y)];
                    if (x > y) v.y = -v.y;
                    return v;
                };
                auto put = [&](int x, int y, Z v) {
                    if (x > y) v.y = -v.y;
                    P[rbx(min(x, y)) + max(x, y)] = v;
                };
                // The update of k_jacobi_round, A' = J_a^H M J_b, written with
                // J = [[c, s], [-s e, c e]] so that each 2 x 2 factor costs two
                // complex products and four real-scaled sums.
                const Z zero{0.0, 0.0};
                const Z m00 = get(pa, pb);
                const Z m01 = qb_ok ? get(pa, qb) : zero;
                const Z m10 = qa_ok ? get(qa, pb) : zero;
                const Z m11 = (qa_ok && qb_ok) ? get(qa, qb) : zero;
                const Z u0 = zmul_f(eb, m01), u1 = zmul_f(eb, m11);
                const Z t00 = zaxpby(rbr.c, m00, -rbr.s, u0), t01 = zaxpby(rbr.s, m00, rbr.c, u0);
                const Z t10 = zaxpby(rbr.c, m10, -rbr.s, u1), t11 = zaxpby(rbr.s, m10, rbr.c, u1);
                const Z v0 = zcmul_f(ea, t10), v1 = zcmul_f(ea, t11);
                put(pa, pb, zaxpby(ra.c, t00, -ra.s, v0));
                if (qb_ok) put(pa, qb, zaxpby(ra.c, t01, -ra.s, v1));
                if (qa_ok) put(qa, pb, zaxpby(ra.s, t00, ra.c, v0));
                if (qa_ok && qb_ok) put(qa, qb, zaxpby(ra.s, t01, ra.c, v1));
            }
            __syncthreads();
        }
        // Off-diagonal and total Frobenius norms (each stored off-diagonal
        // entry stands for two).
        double off = 0.0, tot = 0.0;
        for (int e = t; e < n * (n + 1) / 2; e += kJacobiMidThreads) {
            int x = (int)((2.0 * n + 1.0 - sqrt((2.0 * n + 1.0) * (2.0 * n + 1.0) - 8.0 * e)) * 0.5);
            while (x > 0 && pk_idx(x, x, n) > e) --x;
            while (x + 1 < n && pk_idx(x + 1, x + 1, n) <= e) ++x;
            const Z v = P[e];
            const double mm = v.x * v.x + v.y * v.y;
            if (e == pk_idx(x, x, n)) {
                tot += mm;
            } else {
                off += 2.0 * mm;
                tot += 2.0 * mm;
            }
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if (lane == 0) {
            red[0][wave] = off;
            red[1][wave] = tot;
        }
        __syncthreads();
        if (t == 0) {
            double so = 0.0, st = 0.0;
            for (int i = 0; i < nw; ++i) {
                so += red[0][i];
                st += red[1][i];
            }
            const double o = sqrt(so), tt = sqrt(st);
            int d = 0;   // 0 continue, 1 converged, 2 non-finite
            if (!isfinite(o)) d = 2;
            else if (o <= 1e-15 * tt || (o <= 1e-12 * tt && o >= 0.5 * prev)) d = 1;
            prev = o;
            decide = d;
        }
        __syncthreads();
        const int d = decide;
        __syncthreads();   // decide is rewritten after the next sweep
        if (d == 2) {
            result = -2;
            break;
        }
        if (d == 1) {
            result = sweep + 1;
            break;
        }
    }
    if (n == 1) result = 0;
    for (int j = t; j < n; j += kJacobiMidThreads) {
        const double dj = P[pk_idx(j, j, n)].x;
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double di = P[pk_idx(i, i, n)].x;
            rank += (di < dj) || (di == dj && i < j);
        }
        w[rank] = dj;
        perm[j] = rank;
    }
    if (t == 0) {
        hdr[0] = result;
        hdr[1] = rounds;
    }
}

// Y[i, perm[j]] = V[i, j], V = the product of the recorded rotations
// applied to the identity: one wave per row i, the row in LDS, pair k of a
// round handled by lane k % 64.
constexpr int kRotRowsPerBlock = 4;
__global__ __launch_bounds__(64 * kRotRowsPerBlock) void k_jacobi_apply_rot(const Z *__restrict__ work,
                                                                             int n,
                                                                             Z *__restrict__ Y) {
    __shared__ Z rows[kRotRowsPerBlock][kJacobiMid + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * kRotRowsPerBlock + wv;
    if (i >= n) return;   // whole wave; no workgroup barrier below
    const int m = n + (n & 1), h = m / 2;
    const int *hdr = reinterpret_cast<const int *>(work);
    const int *perm = hdr + 16;
    const Z *rec = work + kMidHead;
    const int rounds = hdr[1];
    Z *row = rows[wv];
    for (int j = lane; j < n; j += 64) row[j] = Z{j == i ? 1.0 : 0.0, 0.0};
    wave_sync();
    // Pairs lane and lane + 64 (h <= 70); their rotations for the next round
    // are loaded while the current one is applied.
    const bool has0 = lane < h, has1 = lane + 64 < h;
    Z cs0{1.0, 0.0}, e0{1.0, 0.0}, cs1{1.0, 0.0}, e1{1.0, 0.0};
    auto fetch = [&](int rd, Z &a0, Z &b0, Z &a1, Z &b1) {
        if (rd >= rounds) return;
        const Z *o = rec + 2 * (int64_t)rd * h;
        if (has0) {
            a0 = o[2 * lane];
            b0 = o[2 * lane + 1];
        }
        if (has1) {
            a1 = o[2 * (lane + 64)];
            b1 = o[2 * (lane + 64) + 1];
        }
    };
    fetch(0, cs0, e0, cs1, e1);
    for (int rd = 0; rd < rounds; ++rd) {
        Z ncs0 = cs0, ne0 = e0, ncs1 = cs1, ne1 = e1;
        fetch(rd + 1, ncs0, ne0, ncs1, ne1);
        const int round = rd % (m - 1);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const bool has = u == 0 ? has0 : has1;
            if (!has) continue;
            const int k = lane + 64 * u;
            const Z cs = u == 0 ? cs0 : cs1, e = u == 0 ? e0 : e1;
            int p, q;
            rr_pair(m, round, k, p, q);
            if (q >= n) continue;
            const Z vp = row[p], vq = row[q];
            const Z j10b = zscale(e, -cs.y), j11b = zscale(e, cs.x);
            row[p] = zadd(zscale(vp, cs.x), zmul(vq, j10b));
            row[q] = zadd(zscale(vp, cs.y), zmul(vq, j11b));
        }
        wave_sync();
        cs0 = ncs0;
        e0 = ne0;
        cs1 = ncs1;
        e1 = ne1;
    }
    for (int j = lane; j < n; j += 64) Y[(int64_t)i * n + perm[j]] = row[j];
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
    const size_t np = chol_np(n);
    return 2 * np * np + (np + 1) / 2 + 1;
}

void chol_qr_factor(const Z *G, int n, double shift, Z *B, Z *work, int *info,
                    hipStream_t s) {
    if (n < 1 || n > 1024) throw Error(7, "chol_qr_factor: order out of range");
    const int nt = (n + 15) / 16;
    hipLaunchKernelGGL(k_chol_prep, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, G, n,
                       shift, B, work);
    check_launch("k_chol_prep");
    hipLaunchKernelGGL(k_chol_blocked, dim3(1), dim3(kCholThreads), 0, s, G, n, B, work, info);
    check_launch("k_chol_blocked");
}

size_t jacobi_work_elems(int n) {
    // The mid-size path's rotation record grows with n up to kJacobiMid;
    // smaller orders than n use it too (locking shrinks the problem).
    size_t e = (size_t)3 * n * n;
    if (n > kJacobiLds) e = std::max(e, jacobi_mid_elems(std::min(n, kJacobiMid)));
    return e;
}

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
    if (n > kJacobiMid) return;   // the sweep path checks as it goes
    if (st == -2) throw Error(5, "jacobi: non-finite matrix");
    if (st == -1) {
        const int cap = n > kJacobiLds ? std::min(jacobi_max_sweeps(), kRotSweeps)
                                       : jacobi_max_sweeps();
        throw Error(7, "jacobi: the reduced eigenproblem did not converge in " +
                           std::to_string(cap) + " sweeps");
    }
}

void jacobi_eig(Z *A, int n, double *w, Z *Y, Z *work, double *hwork,
                hipStream_t s, JacobiGraphs *graphs, int *hstatus) {
    if (n <= kJacobiLds) {
        // One launch, no host round trip per sweep; the status word lives
        // in the (otherwise unused) work buffer.  8 waves at every order: a
        // round's work is what bounds it (n = 30: 1 wave 1057 us, 2 waves
        // 623, 4 waves 380, 8 waves 340 per eigensolve), and no more, so
        // that the launch fits beside other kernels.
        const int max_sweeps = jacobi_max_sweeps();
        int *dstatus = reinterpret_cast<int *>(work);
        const int threads = 512;
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
    if (n <= kJacobiMid) {
        // Two launches, the status word read with the caller's results.
        const int max_sweeps = std::min(jacobi_max_sweeps(), kRotSweeps);
        int *dstatus = reinterpret_cast<int *>(work);
        hipLaunchKernelGGL(k_jacobi_mid, dim3(1), dim3(kJacobiMidThreads), 0, s, (const Z *)A,
                           n, max_sweeps, w, work);
        check_launch("k_jacobi_mid");
        hipLaunchKernelGGL(k_jacobi_apply_rot, dim3((n + kRotRowsPerBlock - 1) / kRotRowsPerBlock),
                           dim3(64 * kRotRowsPerBlock), 0, s, (const Z *)work, n, Y);
        check_launch("k_jacobi_apply_rot");
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
