// Chebyshev filter step as one complex HEMM with the recurrence fused into
// the epilogue:  W = a * H Y + b * Y + g * X   (Filter phase of ChASE).
//
// H is N x N complex128, column-major; Y, X, W are N x n row-major blocks.
// Arithmetic: FP64 MFMA (v_mfma_f64_16x16x4_f64), four real products per
// complex product (no 3M trick, so every product is exact FP64 MFMA work).
//
// Tiling (gfx950):
//  * a workgroup is 4 waves; wave w owns rows [16w, 16w+16) of a 64-row
//    block and 16*WN columns (WN 16x16 complex tiles = 2*WN FP64
//    accumulator tiles);
//  * MFMA operand A (16 rows x 4 k of H) is one 16-byte load per lane,
//    coalesced along the column of H; operand B (4 k x 16 columns of Y) is
//    one 16-byte load per lane per tile, coalesced along the row of Y.
//    Both come straight from L1/L2: at 64 cycles per FP64 MFMA the operand
//    traffic is ~12 B/clk/CU, well inside L1 bandwidth, so no LDS staging;
//  * the four waves of a workgroup read the same Y rows, which L1 serves;
//  * K (the column index of H) can be split into `splits` ranges to balance
//    the tile count over 256 CUs; partial sums are then reduced in a fixed
//    order by a second kernel that also applies the epilogue (deterministic);
//  * XCD-aware tile order: workgroups are dispatched round-robin over the 8
//    XCDs, so all tiles of one 64-row block of H (its column blocks and K
//    splits) are given ids on the same XCD and share that XCD's L2.
#include "common.h"

namespace chase {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int WN, bool FUSED>
__global__ __launch_bounds__(256) void k_filter(
    const Z *__restrict__ H, int64_t ldh, int N, const Z *__restrict__ Y,
    int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
    double b, double g, int rb_count, int cb_count, int splits, int kchunk,
    Z *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;

    const int id = blockIdx.x;
    const int xcd = id & 7;
    const int local = id >> 3;
    const int per = cb_count * splits;
    const int rb = (local / per) * 8 + xcd;
    if (rb >= rb_count) return;
    const int rem = local % per;
    const int cb = rem % cb_count;
    const int sp = rem / cb_count;
    const int row0 = rb * 64 + wave * 16;
    if (row0 >= N) return;
    const int col0 = cb * 16 * WN;
    const int kbeg = sp * kchunk;
    const int kend = min(N, kbeg + kchunk);

    // Rows past N and columns past n are computed on clamped (valid)
    // addresses and never stored.
    const int arow = min(row0 + r, N - 1);
    const Z *hp = H + arow + (int64_t)(kbeg + q) * ldh;
    const int64_t hstep = 4 * ldh;
    int ycol[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) ycol[c] = min(col0 + 16 * c + r, n - 1);
    const Z *yp = Y + (int64_t)(kbeg + q) * ldy;
    const int64_t ystep = 4 * ldy;

    v4d cr[WN], ci[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        cr[c] = v4d{0.0, 0.0, 0.0, 0.0};
        ci[c] = v4d{0.0, 0.0, 0.0, 0.0};
    }

    const int kfull = kbeg + ((kend - kbeg) & ~3);
    int k = kbeg;
    if (k < kfull) {
        // Software pipeline: operands of step k+4 load while step k computes.
        Z h = *hp;
        Z y[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) y[c] = yp[ycol[c]];
        for (; k + 4 < kfull; k += 4) {
            hp += hstep;
            yp += ystep;
            Z hn = *hp;
            Z yn[WN];
#pragma unroll
            for (int c = 0; c < WN; ++c) yn[c] = yp[ycol[c]];
            const double nhy = -h.y;
#pragma unroll
            for (int c = 0; c < WN; ++c) cr[c] = mfma64(h.x, y[c].x, cr[c]);
#pragma unroll
            for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.x, y[c].y, ci[c]);
#pragma unroll
            for (int c = 0; c < WN; ++c) cr[c] = mfma64(nhy, y[c].y, cr[c]);
#pragma unroll
            for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.y, y[c].x, ci[c]);
            h = hn;
#pragma unroll
            for (int c = 0; c < WN; ++c) y[c] = yn[c];
        }
        const double nhy = -h.y;
#pragma unroll
        for (int c = 0; c < WN; ++c) cr[c] = mfma64(h.x, y[c].x, cr[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.x, y[c].y, ci[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) cr[c] = mfma64(nhy, y[c].y, cr[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.y, y[c].x, ci[c]);
        hp += hstep;
        yp += ystep;
        k = kfull;
    }
    if (k < kend) {
        // Ragged tail of K: lanes whose k is past the end contribute zero
        // and do not load.
        const bool ok = (k + q) < kend;
        Z h = ok ? *hp : Z{0.0, 0.0};
        Z y[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) y[c] = ok ? yp[ycol[c]] : Z{0.0, 0.0};
        const double nhy = -h.y;
#pragma unroll
        for (int c = 0; c < WN; ++c) cr[c] = mfma64(h.x, y[c].x, cr[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.x, y[c].y, ci[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) cr[c] = mfma64(nhy, y[c].y, cr[c]);
#pragma unroll
        for (int c = 0; c < WN; ++c) ci[c] = mfma64(h.y, y[c].x, ci[c]);
    }

    // Accumulator layout of the 16x16 FP64 MFMA: lane (r, q) holds rows
    // q, q+4, q+8, q+12 of column r (register v holds row q + 4v).
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        const int col = col0 + 16 * c + r;
        if (col >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + q + 4 * v;
            if (row >= N) continue;
            const double sr = cr[c][v], si = ci[c][v];
            if (FUSED) {
                const Z yv = Y[(int64_t)row * ldy + col];
                Z o;
                o.x = a * sr + b * yv.x;
                o.y = a * si + b * yv.y;
                if (g != 0.0) {
                    const Z xv = X[(int64_t)row * ldx + col];
                    o.x += g * xv.x;
                    o.y += g * xv.y;
                }
                W[(int64_t)row * ldw + col] = o;
            } else {
                part[((int64_t)sp * N + row) * n + col] = Z{sr, si};
            }
        }
    }
}

// Ordered sum of the split-K partials plus the recurrence epilogue.
__global__ __launch_bounds__(256) void k_filter_reduce(
    const Z *__restrict__ part, int splits, int N, int n, const Z *Y,
    int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, double a,
    double b, double g) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / n;
        const int col = (int)(t - row * n);
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < splits; ++s) {
            const Z p = part[(int64_t)s * total + t];
            sr += p.x;
            si += p.y;
        }
        const Z yv = Y[row * ldy + col];
        Z o;
        o.x = a * sr + b * yv.x;
        o.y = a * si + b * yv.y;
        if (g != 0.0) {
            const Z xv = X[row * ldx + col];
            o.x += g * xv.x;
            o.y += g * xv.y;
        }
        W[row * ldw + col] = o;
    }
}

template <int WN>
void launch_wn(const FilterPlan &p, const Z *H, int64_t ldh, int N, const Z *Y,
               int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n,
               double a, double b, double g, Z *part, hipStream_t s) {
    const int groups = (p.rb + 7) / 8;
    const int nblocks = groups * 8 * p.cb * p.splits;
    if (p.splits == 1) {
        hipLaunchKernelGGL((k_filter<WN, true>), dim3(nblocks), dim3(256), 0, s,
                           H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, p.rb,
                           p.cb, 1, p.kchunk, nullptr);
    } else {
        hipLaunchKernelGGL((k_filter<WN, false>), dim3(nblocks), dim3(256), 0,
                           s, H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g,
                           p.rb, p.cb, p.splits, p.kchunk, part);
    }
}

}  // namespace

FilterPlan filter_plan(int64_t N, int n) {
    FilterPlan p{};
    const int nb16 = (n + 15) / 16;
    if (nb16 <= 10) {
        p.cb = 1;
        p.wn = nb16;
    } else {
        p.cb = (nb16 + 9) / 10;
        p.wn = (nb16 + p.cb - 1) / p.cb;
    }
    p.rb = (int)((N + 63) / 64);
    // Balance: workgroup slots ~ 256 CUs x (2 resident workgroups when the
    // accumulators leave room for two waves per SIMD).
    const int64_t slots = 256 * (p.wn <= 8 ? 2 : 1);
    const int64_t units = (int64_t)p.rb * p.cb;
    const int cand[] = {1, 2, 3, 4, 6, 8};
    double best = 1e300;
    int bests = 1;
    for (int sp : cand) {
        if (sp > 1 && N / sp < 1024) break;
        const double rounds = (double)((units * sp + slots - 1) / slots);
        const double cost = rounds / sp * (1.0 + 0.01 * (sp - 1));
        if (cost < best * 0.97) {
            best = cost;
            bests = sp;
        }
    }
    p.splits = bests;
    int64_t kc = (N + p.splits - 1) / p.splits;
    kc = (kc + 3) & ~int64_t(3);
    p.kchunk = (int)kc;
    return p;
}

size_t filter_partial_elems(int64_t N, int n) {
    const FilterPlan p = filter_plan(N, n);
    return p.splits > 1 ? (size_t)p.splits * (size_t)N * (size_t)n : 0;
}

void filter_gemm(const Z *H, int64_t ldh, int64_t N64, const Z *Y, int64_t ldy,
                 const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
                 double b, double g, Z *part, hipStream_t s,
                 hipEvent_t after_mfma) {
    if (n <= 0 || N64 <= 0) return;
    const int N = (int)N64;
    const FilterPlan p = filter_plan(N64, n);
    if (p.splits > 1 && !part) throw Error(7, "filter_gemm: missing partials");
    switch (p.wn) {
#define CASE(w) \
    case w: launch_wn<w>(p, H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, part, s); break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: throw Error(7, "filter_gemm: bad tile width");
    }
    check_launch("k_filter");
    if (after_mfma) CHASE_HIP(hipEventRecord(after_mfma, s));
    if (p.splits > 1) {
        const int64_t total = (int64_t)N * n;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_filter_reduce, dim3(blocks), dim3(256), 0, s, part,
                           p.splits, N, n, Y, ldy, X, ldx, W, ldw, a, b, g);
        check_launch("k_filter_reduce");
    }
}

}  // namespace chase
