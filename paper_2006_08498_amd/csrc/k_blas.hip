// Tall-skinny products, reductions and layout kernels used by the QR, RR,
// Resid and Lanczos phases.  Blocks are row-major N x n (element (i, j) at
// p[i*ld + j]); every reduction has a fixed order (no atomics), so results
// are bitwise reproducible.
#include "common.h"

#include <algorithm>

namespace chase {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ gram
// part[s] (p x q) = sum over rows of chunk s of conj(A[i, :])^T B[i, :].
// Workgroup = 4 waves over interleaved 4-row steps of the chunk, one
// 16 x 16*WN tile of C; the four wave sums are added in LDS in wave order.
// Each wave keeps kGramDepth steps' operands in flight (registers), so the
// loads of later steps overlap the products of the current one.
// herm (A = B, p = q, a Hermitian result): only the tiles that reach the
// diagonal or above are launched (active(jb) = min(pb, (jb + 1) WN) row
// tiles in column tile jb); the partial sums fill the rest from their
// mirror images.
constexpr int kGramDepth = 4;

template <int WN>
__global__ __launch_bounds__(256) void k_gram(const Z *__restrict__ A,
                                              int64_t lda,
                                              const Z *__restrict__ B,
                                              int64_t ldb, int N, int p, int q,
                                              int pb, int qb, int tiles, int chunk,
                                              int nchunks, Z *__restrict__ part, int herm) {
    __shared__ double red[3][64 * 8 * WN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, qq = lane >> 4;
    // XCD-aware order: workgroup b runs on XCD b % 8, and every tile of
    // chunk s is placed on XCD s % 8, so the chunk's rows come from HBM
    // once and are re-read from that XCD's L2.
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int tile = slot % tiles, s = xcd + 8 * (slot / tiles);
    if (s >= nchunks) return;   // padding of the chunk count to a multiple of 8
    int ib, jb;
    if (!herm) {
        ib = tile % pb;
        jb = tile / pb;
    } else {
        jb = 0;
        int rest = tile;
        while (rest >= min(pb, (jb + 1) * WN)) {
            rest -= min(pb, (jb + 1) * WN);
            ++jb;
        }
        ib = rest;
    }
    const int p0 = ib * 16, q0 = jb * 16 * WN;
    const int kbeg = s * chunk, kend = min(N, kbeg + chunk);
    const int acol = min(p0 + r, p - 1);
    int bcol[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) bcol[c] = min(q0 + 16 * c + r, q - 1);
    v4d cr[WN], ci[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        cr[c] = v4d{0, 0, 0, 0};
        ci[c] = v4d{0, 0, 0, 0};
    }
    // Step operands: rows past the chunk read row kbeg and count as zero.
    Z abuf[kGramDepth], bbuf[kGramDepth][WN];
    bool okb[kGramDepth];
    auto load = [&](int k, int d) {
        const int row = k + qq;
        okb[d] = row < kend;
        const int64_t rr = okb[d] ? row : kbeg;
        abuf[d] = A[rr * lda + acol];
#pragma unroll
        for (int c = 0; c < WN; ++c) bbuf[d][c] = B[rr * ldb + bcol[c]];
    };
    const int k0 = kbeg + 4 * wave;
#pragma unroll
    for (int d = 0; d < kGramDepth; ++d) load(k0 + 16 * d, d);
    for (int k = k0; k < kend; k += 16 * kGramDepth) {
#pragma unroll
        for (int d = 0; d < kGramDepth; ++d) {
            const Z a = okb[d] ? abuf[d] : Z{0.0, 0.0};
            const double nay = -a.y;
#pragma unroll
            for (int c = 0; c < WN; ++c) {
                const Z bv = bbuf[d][c];
                cr[c] = mfma64(a.x, bv.x, cr[c]);
                ci[c] = mfma64(a.x, bv.y, ci[c]);
                cr[c] = mfma64(a.y, bv.y, cr[c]);
                ci[c] = mfma64(nay, bv.x, ci[c]);
            }
            load(k + 16 * (d + kGramDepth), d);
        }
    }
    // Fixed-order sum of the four waves' tiles.
    if (wave > 0) {
#pragma unroll
        for (int c = 0; c < WN; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                red[wave - 1][(c * 8 + v) * 64 + lane] = cr[c][v];
                red[wave - 1][(c * 8 + 4 + v) * 64 + lane] = ci[c][v];
            }
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int c = 0; c < WN; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    cr[c][v] += red[w][(c * 8 + v) * 64 + lane];
                    ci[c][v] += red[w][(c * 8 + 4 + v) * 64 + lane];
                }
#pragma unroll
        for (int c = 0; c < WN; ++c) {
            const int col = q0 + 16 * c + r;
            if (col >= q) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = p0 + qq + 4 * v;   // FP64 MFMA: register v holds row qq + 4v
                if (row >= p) continue;
                part[((int64_t)s * p + row) * q + col] = Z{cr[c][v], ci[c][v]};
            }
        }
    }
}

// C = sum of the partials in a fixed order: a workgroup owns 64 entries,
// wave w sums partials w, w + 4, ... and the four sums are added in wave
// order.  herm: only the entries on and above the diagonal are summed;
// each sets its mirror to the conjugate and a diagonal entry is made real,
// so C is Hermitian to the last bit.
__global__ __launch_bounds__(256) void k_sum_parts(const Z *__restrict__ part, int nparts,
                                                   int p, int q, Z *__restrict__ C,
                                                   int64_t ldc, int herm) {
    __shared__ Z red[3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t total = (int64_t)p * q;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const int64_t tc = t < total ? t : 0;
    const int64_t i = tc / q, j = tc - i * q;
    const bool skip = herm && i > j;   // uniform per entry across the waves
    double sr = 0.0, si = 0.0;
    if (!skip) {
        int sidx = wave;
        for (; sidx + 12 < nparts; sidx += 16) {
            Z v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)(sidx + 4 * u) * total + tc];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sr += v[u].x;
                si += v[u].y;
            }
        }
        for (; sidx < nparts; sidx += 4) {
            const Z v = part[(int64_t)sidx * total + tc];
            sr += v.x;
            si += v.y;
        }
    }
    if (wave > 0) red[wave - 1][lane] = Z{sr, si};
    __syncthreads();
    if (wave != 0 || t >= total || skip) return;
    for (int w = 0; w < 3; ++w) {
        sr += red[w][lane].x;
        si += red[w][lane].y;
    }
    if (!herm) {
        C[i * ldc + j] = Z{sr, si};
    } else if (i == j) {
        C[i * ldc + j] = Z{sr, 0.0};
    } else {
        C[i * ldc + j] = Z{sr, si};
        C[j * ldc + i] = Z{sr, -si};
    }
}

struct GramPlan {
    int wn, pb, qb, tiles, chunks, chunk;
};

GramPlan gram_plan(int64_t N, int p, int q, bool herm) {
    GramPlan g{};
    const int nb = (q + 15) / 16;
    g.qb = (nb + 3) / 4;   // at most 4 tiles per wave (LDS: 48 KiB)
    g.wn = (nb + g.qb - 1) / g.qb;
    g.pb = (p + 15) / 16;
    g.tiles = g.pb * g.qb;
    if (herm) {
        g.tiles = 0;
        for (int jb = 0; jb < g.qb; ++jb) g.tiles += std::min(g.pb, (jb + 1) * g.wn);
    }
    int64_t want = (1024 + g.tiles - 1) / g.tiles;
    int64_t maxc = (N + 255) / 256;
    g.chunks = (int)std::max<int64_t>(1, std::min(want, maxc));
    int64_t ch = (N + g.chunks - 1) / g.chunks;
    ch = (ch + 15) & ~int64_t(15);
    g.chunk = (int)ch;
    g.chunks = (int)((N + ch - 1) / ch);
    // Chunk s runs on XCD s mod 8: a count that is not a multiple of 8
    // leaves some XCDs a chunk more than the rest (10 chunks at n = 400 gave
    // two XCDs twice the work of the other six), so round it up.
    if (g.chunks > 8 && g.chunks % 8) {
        const int64_t c8 = (g.chunks + 7) / 8 * 8;
        ch = (N + c8 - 1) / c8;
        ch = (ch + 15) & ~int64_t(15);
        g.chunk = (int)ch;
        g.chunks = (int)((N + ch - 1) / ch);
    }
    return g;
}

template <int WN>
void launch_gram(const GramPlan &g, const Z *A, int64_t lda, const Z *B,
                 int64_t ldb, int N, int p, int q, Z *part, int herm, hipStream_t s) {
    const int blocks = g.tiles * ((g.chunks + 7) / 8 * 8);
    hipLaunchKernelGGL(k_gram<WN>, dim3(blocks), dim3(256), 0, s, A, lda, B,
                       ldb, N, p, q, g.pb, g.qb, g.tiles, g.chunk, g.chunks, part, herm);
}

// ------------------------------------------------------------------ tsmm
// C (N x q) = alpha * A (N x p) B (p x q) + beta * C0; wave = 16 rows x
// 16*WN columns, K = p.
// upper: B is upper triangular, so a column block's sum stops at its last
// column (the rows below are zero).
template <int WN>
__global__ __launch_bounds__(256) void k_tsmm(
    const Z *__restrict__ A, int64_t lda, const Z *__restrict__ B, int64_t ldb,
    int N, int p, int q, double alpha, const Z *C0, int64_t ldc0, double beta,
    Z *C, int64_t ldc, int cb, int upper) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, qq = lane >> 4;
    // XCD-aware order: workgroup b runs on XCD b % 8; the column blocks of
    // row block rbk share XCD rbk % 8, so A's rows are re-read from its L2.
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int rbk = xcd + 8 * (slot / cb), cbk = slot % cb;
    const int row0 = rbk * 64 + wave * 16;
    if (row0 >= N) return;
    const int col0 = cbk * 16 * WN;
    const int arow = min(row0 + r, N - 1);
    const Z *ap = A + (int64_t)arow * lda;
    int bcol[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) bcol[c] = min(col0 + 16 * c + r, q - 1);
    v4d cr[WN], ci[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        cr[c] = v4d{0, 0, 0, 0};
        ci[c] = v4d{0, 0, 0, 0};
    }
    const int kmax = upper ? min(p, col0 + 16 * WN) : p;
    // Step operands, D steps in flight; steps past kmax read
    // k = 0 and count as zero.
    constexpr int D = WN <= 4 ? 4 : 2;
    Z abuf[D], bbuf[D][WN];
    bool okb[D];
    auto load = [&](int k, int d) {
        const int kk = k + qq;
        okb[d] = kk < kmax;
        const int kc = okb[d] ? kk : 0;
        abuf[d] = ap[kc];
#pragma unroll
        for (int c = 0; c < WN; ++c) bbuf[d][c] = B[(int64_t)kc * ldb + bcol[c]];
    };
    if (kmax > 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) load(4 * d, d);
    }
    for (int k = 0; k < kmax; k += 4 * D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const Z a = okb[d] ? abuf[d] : Z{0.0, 0.0};
            const double nay = -a.y;
#pragma unroll
            for (int c = 0; c < WN; ++c) {
                const Z bv = bbuf[d][c];
                cr[c] = mfma64(a.x, bv.x, cr[c]);
                ci[c] = mfma64(a.x, bv.y, ci[c]);
                cr[c] = mfma64(nay, bv.y, cr[c]);
                ci[c] = mfma64(a.y, bv.x, ci[c]);
            }
            load(k + 4 * (d + D), d);
        }
    }
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        const int col = col0 + 16 * c + r;
        if (col >= q) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + qq + 4 * v;   // FP64 MFMA: register v holds row qq + 4v
            if (row >= N) continue;
            Z o{alpha * cr[c][v], alpha * ci[c][v]};
            if (beta != 0.0) {
                const Z z = C0[(int64_t)row * ldc0 + col];
                o.x += beta * z.x;
                o.y += beta * z.y;
            }
            C[(int64_t)row * ldc + col] = o;
        }
    }
}

// ------------------------------------------------------------ col norms
// part[blk][j] = sum_{i in blk} |V[i,j] - theta_j V2[i,j]|^2
__global__ __launch_bounds__(256) void k_colnorm_part(
    const Z *__restrict__ V, int64_t ldv, const Z *__restrict__ V2,
    int64_t ldv2, const double *__restrict__ theta, int N, int n, int rows,
    double *__restrict__ part) {
    const int blk = blockIdx.x;
    const int i0 = blk * rows, i1 = min(N, i0 + rows);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double acc = 0.0;
        const double th = V2 ? theta[j] : 0.0;
        for (int i = i0; i < i1; ++i) {
            Z v = V[(int64_t)i * ldv + j];
            if (V2) {
                const Z u = V2[(int64_t)i * ldv2 + j];
                v.x -= th * u.x;
                v.y -= th * u.y;
            }
            acc += v.x * v.x + v.y * v.y;
        }
        part[(int64_t)blk * n + j] = acc;
    }
}

// One wave per column: lanes take strided partials, then a butterfly sum
// (a fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void k_colnorm_final(const double *__restrict__ part,
                                                       int nblk, int n,
                                                       double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= n) return;   // uniform per wave
    double acc = 0.0;
    for (int b = lane; b < nblk; b += 64) acc += part[(int64_t)b * n + j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) out[j] = sqrt(acc);
}

int norm_blocks(int64_t N) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (N + 63) / 64));
}

// ------------------------------------------------------------ layouts
__global__ void k_copy(const Z *__restrict__ src, int64_t lds, Z *dst,
                       int64_t ldd, int N, int n) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        dst[i * ldd + j] = src[i * lds + j];
    }
}

__global__ void k_permute(const Z *__restrict__ src, int64_t lds,
                          Z *__restrict__ dst, int64_t ldd, int N, int n,
                          const int *__restrict__ perm) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        dst[i * ldd + j] = src[i * lds + perm[j]];
    }
}

// 32 x 32 tiles through LDS so both sides are coalesced.
__global__ __launch_bounds__(256) void k_c2r(const Z *__restrict__ src,
                                             int64_t ldc, Z *__restrict__ dst,
                                             int64_t ldr, int N, int n) {
    __shared__ Z tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int jj = ty; jj < 32; jj += 8) {
        const int i = i0 + tx, j = j0 + jj;
        if (i < N && j < n) tile[jj][tx] = src[i + (int64_t)j * ldc];
    }
    __syncthreads();
    for (int ii = ty; ii < 32; ii += 8) {
        const int i = i0 + ii, j = j0 + tx;
        if (i < N && j < n) dst[(int64_t)i * ldr + j] = tile[tx][ii];
    }
}

__global__ __launch_bounds__(256) void k_r2c(const Z *__restrict__ src,
                                             int64_t ldr, Z *__restrict__ dst,
                                             int64_t ldc, int N, int n,
                                             const Z *__restrict__ phase) {
    __shared__ Z tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int ii = ty; ii < 32; ii += 8) {
        const int i = i0 + ii, j = j0 + tx;
        if (i < N && j < n) tile[ii][tx] = src[(int64_t)i * ldr + j];
    }
    __syncthreads();
    for (int jj = ty; jj < 32; jj += 8) {
        const int i = i0 + tx, j = j0 + jj;
        if (i < N && j < n) {
            Z v = tile[tx][jj];
            if (phase) {
                const Z ph = phase[j];   // (conj(v_max)/|v_max|, index)
                const Z o{v.x * ph.x - v.y * ph.y, v.x * ph.y + v.y * ph.x};
                v = o;
                if ((double)i == phase[n + j].x) v.y = 0.0;
            }
            dst[i + (int64_t)j * ldc] = v;
        }
    }
}

// Largest |v_ij|^2 per column (lowest index on ties), two passes.
__global__ __launch_bounds__(256) void k_absmax_part(
    const Z *__restrict__ V, int64_t ldv, int N, int n, int rows,
    double *__restrict__ part) {
    const int blk = blockIdx.x;
    const int i0 = blk * rows, i1 = min(N, i0 + rows);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double best = -1.0, bi = 0.0;
        for (int i = i0; i < i1; ++i) {
            const Z v = V[(int64_t)i * ldv + j];
            const double m = v.x * v.x + v.y * v.y;
            if (m > best) {
                best = m;
                bi = i;
            }
        }
        part[((int64_t)blk * n + j) * 2] = best;
        part[((int64_t)blk * n + j) * 2 + 1] = bi;
    }
}

// phase[j] = conj(v_max)/|v_max|, phase[n + j].x = row of v_max.
__global__ void k_absmax_final(const double *__restrict__ part, int nblk,
                               const Z *__restrict__ V, int64_t ldv, int n,
                               Z *__restrict__ phase) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double best = -1.0, bi = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double m = part[((int64_t)b * n + j) * 2];
        if (m > best) {
            best = m;
            bi = part[((int64_t)b * n + j) * 2 + 1];
        }
    }
    const Z v = V[(int64_t)bi * ldv + j];
    const double a = sqrt(v.x * v.x + v.y * v.y);
    phase[j] = a > 0.0 ? Z{v.x / a, -v.y / a} : Z{1.0, 0.0};
    phase[n + j] = Z{bi, 0.0};
}

// ------------------------------------------------------------ random
// Philox4x32-10 (Salmon et al., SC'11): round multipliers 0xD2511F53,
// 0xCD9E8D57, key increments 0x9E3779B9, 0xBB67AE85.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0,
                                         uint32_t k1) {
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) *
           (1.0 / 9007199254740992.0);
}

__global__ void k_random(Z *V, int64_t ld, int N, int n, uint32_t k0,
                         uint32_t k1, uint32_t stream) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        uint32_t c[4] = {(uint32_t)i, (uint32_t)j, stream, 0u};
        philox10(c, k0, k1);
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        const double s = 0.70710678118654752440;
        V[i * ld + j] = Z{rad * cs * s, rad * sn * s};
    }
}

__global__ void k_check_finite(const Z *__restrict__ H, int64_t ldh, int N,
                               int *flag) {
    const int64_t total = (int64_t)N * N;
    int bad = 0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / N, i = t - j * N;
        const Z v = H[i + j * ldh];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    }
    if (bad) *flag = 1;   // every writer stores the same value
}

// ------------------------------------------------------------ Lanczos
// One workgroup per run (column `run` of the row-major N x r blocks).
template <int NT>
__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

// Lanczos vector update for r independent runs (columns of N x r
// row-major blocks v, vp, w), in three launches over a grid of blocks x
// runs; partial sums go to `part` (2 * blocks * r doubles) and every block
// reduces them in the same fixed order:
//   dot:    part[run][b] = Re(v^H w) over the block's rows;
//   update: alpha = sum; w -= alpha v + beta_prev vp; part2 = |w|^2 partial;
//   scale:  beta = sqrt(sum); vp = v; v = w / beta.
// The first step (normalise_only) skips dot and update: v = w / |w|, vp = 0.
constexpr int kLzThreads = 256;

__device__ double lz_sum_parts(const double *p, int nb, double *sh) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kLzThreads) acc += p[b];
    return block_sum<kLzThreads>(acc, sh);
}

__global__ __launch_bounds__(kLzThreads) void k_lz_dot(const Z *v, const Z *w, int64_t ld,
                                                       int N, int rows, double *part) {
    __shared__ double sh[kLzThreads];
    const int b = blockIdx.x, run = blockIdx.y, nb = gridDim.x;
    const int i1 = min(N, (b + 1) * rows);
    double s = 0.0;
    for (int i = b * rows + threadIdx.x; i < i1; i += kLzThreads) {
        const Z a = v[(int64_t)i * ld + run], c = w[(int64_t)i * ld + run];
        s += a.x * c.x + a.y * c.y;     // Re(conj(v) w)
    }
    s = block_sum<kLzThreads>(s, sh);
    if (threadIdx.x == 0) part[(int64_t)run * nb + b] = s;
}

__global__ __launch_bounds__(kLzThreads) void k_lz_update(const Z *v, const Z *vp, Z *w,
                                                          int64_t ld, int N, int rows,
                                                          const double *part, double *part2,
                                                          const double *beta_prev,
                                                          int normalise_only) {
    __shared__ double sh[kLzThreads];
    const int b = blockIdx.x, run = blockIdx.y, nb = gridDim.x;
    const double al = normalise_only ? 0.0 : lz_sum_parts(part + (int64_t)run * nb, nb, sh);
    const double bp = (normalise_only || !beta_prev) ? 0.0 : beta_prev[run];
    const int i1 = min(N, (b + 1) * rows);
    double s = 0.0;
    for (int i = b * rows + threadIdx.x; i < i1; i += kLzThreads) {
        const int64_t o = (int64_t)i * ld + run;
        Z c = w[o];
        if (!normalise_only) {
            const Z a = v[o], d = vp[o];
            c.x -= al * a.x + bp * d.x;
            c.y -= al * a.y + bp * d.y;
            w[o] = c;
        }
        s += c.x * c.x + c.y * c.y;
    }
    s = block_sum<kLzThreads>(s, sh);
    if (threadIdx.x == 0) part2[(int64_t)run * nb + b] = s;
}

__global__ __launch_bounds__(kLzThreads) void k_lz_scale(Z *v, Z *vp, const Z *w, int64_t ld,
                                                         int N, int rows, const double *part,
                                                         const double *part2, double *alpha,
                                                         double *beta, int normalise_only) {
    __shared__ double sh[kLzThreads];
    const int b = blockIdx.x, run = blockIdx.y, nb = gridDim.x;
    const double be = sqrt(lz_sum_parts(part2 + (int64_t)run * nb, nb, sh));
    const double inv = be > 0.0 ? 1.0 / be : 0.0;
    const int i1 = min(N, (b + 1) * rows);
    for (int i = b * rows + threadIdx.x; i < i1; i += kLzThreads) {
        const int64_t o = (int64_t)i * ld + run;
        const Z c = w[o];
        vp[o] = normalise_only ? Z{0.0, 0.0} : v[o];
        v[o] = Z{c.x * inv, c.y * inv};
    }
    if (!normalise_only && b == 0) {
        const double al = lz_sum_parts(part + (int64_t)run * nb, nb, sh);
        if (threadIdx.x == 0) {
            alpha[run] = al;
            beta[run] = be;
        }
    }
}

int lz_blocks(int64_t N) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(128, (N + 1023) / 1024));
}

inline int grid_for(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
}

}  // namespace

size_t gram_partial_elems(int64_t N, int p, int q) {
    int chunks = gram_plan(N, p, q, false).chunks;
    if (p == q) chunks = std::max(chunks, gram_plan(N, p, q, true).chunks);
    return (size_t)chunks * (size_t)p * (size_t)q;
}

void gram(const Z *A, int64_t lda, const Z *B, int64_t ldb, int64_t N64, int p,
          int q, Z *C, int64_t ldc, Z *part, hipStream_t s, bool herm) {
    if (p <= 0 || q <= 0) return;
    if (herm && (A != B || lda != ldb || p != q))
        throw Error(7, "gram: a Hermitian product needs A = B");
    const int N = (int)N64;
    const GramPlan g = gram_plan(N64, p, q, herm);
    switch (g.wn) {
#define CASE(w) case w: launch_gram<w>(g, A, lda, B, ldb, N, p, q, part, herm ? 1 : 0, s); break;
        CASE(1) CASE(2) CASE(3) CASE(4)
#undef CASE
        default: throw Error(7, "gram: bad tile width");
    }
    check_launch("k_gram");
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)(((int64_t)p * q + 63) / 64)), dim3(256),
                       0, s, part, g.chunks, p, q, C, ldc, herm ? 1 : 0);
    check_launch("k_sum_parts");
}

void tsmm(const Z *A, int64_t lda, const Z *B, int64_t ldb, int64_t N64, int p,
          int q, double alpha, const Z *C0, int64_t ldc0, double beta, Z *C,
          int64_t ldc, hipStream_t s, bool upper) {
    if (N64 <= 0 || q <= 0) return;
    const int N = (int)N64;
    const int nb = (q + 15) / 16;
    // Upper triangular B: narrow column blocks keep each block's K close to
    // its own columns (16-column blocks do the triangle's work plus the
    // diagonal blocks; 80-column blocks did 1.8 times that at q = 140);
    // 32-column blocks beyond 256 columns keep A's re-reads down.
    const int cb = upper ? (nb <= 16 ? nb : (nb + 1) / 2) : (nb + 7) / 8;
    const int wn = (nb + cb - 1) / cb;
    const int rb = (N + 63) / 64;
    const dim3 grid((rb + 7) / 8 * 8 * cb);   // row blocks past N return at once
    switch (wn) {
#define CASE(w)                                                                \
    case w:                                                                    \
        hipLaunchKernelGGL(k_tsmm<w>, grid, dim3(256), 0, s, A, lda, B, ldb, N, \
                           p, q, alpha, C0, ldc0, beta, C, ldc, cb, upper ? 1 : 0); \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: throw Error(7, "tsmm: bad tile width");
    }
    check_launch("k_tsmm");
}

size_t norm_partial_elems(int64_t N, int n) {
    return (size_t)norm_blocks(N) * (size_t)n * 2;
}

void col_norms(const Z *V, int64_t ldv, const Z *V2, int64_t ldv2,
               const double *theta, int64_t N, int n, double *part,
               double *out, hipStream_t s) {
    if (n <= 0) return;
    const int nblk = norm_blocks(N);
    const int rows = (int)((N + nblk - 1) / nblk);
    hipLaunchKernelGGL(k_colnorm_part, dim3(nblk), dim3(256), 0, s, V, ldv, V2,
                       ldv2, theta, (int)N, n, rows, part);
    check_launch("k_colnorm_part");
    hipLaunchKernelGGL(k_colnorm_final, dim3((n + 3) / 4), dim3(256), 0, s,
                       part, nblk, n, out);
    check_launch("k_colnorm_final");
}

void copy_block(const Z *src, int64_t lds, Z *dst, int64_t ldd, int64_t N,
                int n, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N * n)), dim3(256), 0, s, src, lds,
                       dst, ldd, (int)N, n);
    check_launch("k_copy");
}

void permute_cols(const Z *src, int64_t lds, Z *dst, int64_t ldd, int64_t N,
                  int n, const int *perm, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_permute, dim3(grid_for(N * n)), dim3(256), 0, s, src,
                       lds, dst, ldd, (int)N, n, perm);
    check_launch("k_permute");
}

void colmajor_to_rowmajor(const Z *src, int64_t ldc, Z *dst, int64_t ldr,
                          int64_t N, int n, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    const dim3 grid((unsigned)((N + 31) / 32), (unsigned)((n + 31) / 32));
    hipLaunchKernelGGL(k_c2r, grid, dim3(256), 0, s, src, ldc, dst, ldr, (int)N,
                       n);
    check_launch("k_c2r");
}

void rowmajor_to_colmajor(const Z *src, int64_t ldr, Z *dst, int64_t ldc,
                          int64_t N, int n, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    const dim3 grid((unsigned)((N + 31) / 32), (unsigned)((n + 31) / 32));
    hipLaunchKernelGGL(k_r2c, grid, dim3(256), 0, s, src, ldr, dst, ldc, (int)N,
                       n, (const Z *)nullptr);
    check_launch("k_r2c");
}

size_t phase_scratch_elems(int64_t N, int n) {
    // absmax partials (2 doubles per block and column) + 2n complex phases
    return (size_t)norm_blocks(N) * (size_t)n * 2 + (size_t)n * 4;
}

void phase_normalise_out(const Z *V, int64_t ldv, int64_t N, int n, Z *dst,
                         int64_t ldd, double *scratch, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    const int nblk = norm_blocks(N);
    const int rows = (int)((N + nblk - 1) / nblk);
    double *part = scratch;
    Z *phase = reinterpret_cast<Z *>(scratch + (size_t)nblk * n * 2);
    hipLaunchKernelGGL(k_absmax_part, dim3(nblk), dim3(256), 0, s, V, ldv,
                       (int)N, n, rows, part);
    check_launch("k_absmax_part");
    hipLaunchKernelGGL(k_absmax_final, dim3((n + 255) / 256), dim3(256), 0, s,
                       part, nblk, V, ldv, n, phase);
    check_launch("k_absmax_final");
    const dim3 grid((unsigned)((N + 31) / 32), (unsigned)((n + 31) / 32));
    hipLaunchKernelGGL(k_r2c, grid, dim3(256), 0, s, V, ldv, dst, ldd, (int)N,
                       n, (const Z *)phase);
    check_launch("k_r2c");
}

void random_block(Z *V, int64_t ld, int64_t N, int n, uint64_t seed,
                  uint32_t stream, hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_random, dim3(grid_for(N * n)), dim3(256), 0, s, V, ld,
                       (int)N, n, (uint32_t)seed, (uint32_t)(seed >> 32),
                       stream);
    check_launch("k_random");
}

void check_finite(const Z *H, int64_t ldh, int64_t N, int *flag,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(N * N)), dim3(256), 0, s,
                       H, ldh, (int)N, flag);
    check_launch("k_check_finite");
}

size_t lanczos_scratch_elems(int64_t N, int r) { return (size_t)2 * lz_blocks(N) * r; }

void lanczos_update(Z *v, Z *vp, Z *w, int64_t ld, int64_t N, int r,
                    double *alpha, double *beta, int step, int normalise_only,
                    double *scratch, hipStream_t s) {
    const int nb = lz_blocks(N);
    const int rows = (int)((N + nb - 1) / nb);
    double *part = scratch, *part2 = scratch + (size_t)nb * r;
    const dim3 grid(nb, r);
    if (!normalise_only) {
        hipLaunchKernelGGL(k_lz_dot, grid, dim3(kLzThreads), 0, s, v, w, ld, (int)N, rows, part);
        check_launch("k_lz_dot");
    }
    const double *bprev = step > 0 ? beta + (size_t)(step - 1) * r : nullptr;
    hipLaunchKernelGGL(k_lz_update, grid, dim3(kLzThreads), 0, s, v, vp, w, ld, (int)N, rows,
                       part, part2, bprev, normalise_only);
    check_launch("k_lz_update");
    hipLaunchKernelGGL(k_lz_scale, grid, dim3(kLzThreads), 0, s, v, vp, w, ld, (int)N, rows,
                       part, part2, alpha + (size_t)step * r, beta + (size_t)step * r,
                       normalise_only);
    check_launch("k_lz_scale");
}

}  // namespace chase
