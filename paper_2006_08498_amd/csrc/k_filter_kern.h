// Filter GEMM kernel template, shared by the two translation units that
// instantiate it (k_filter.hip: tile widths 1-8, built with the VGPR form of
// MFMA; k_filter_wide.hip: widths 9-10, built with the AGPR form).  The
// register allocator keeps the accumulators in place only with the right
// form for each width (otherwise it moves them between register files every
// k step).
#pragma once

#include "common.h"

namespace chase {
namespace filter_detail {


typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int WN, int PD, bool FUSED>
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
    const int kend = max(kbeg, min(N, kbeg + kchunk));

    // Rows past N and columns past n are computed on clamped (valid)
    // addresses and never stored.
    const int arow = min(row0 + r, N - 1);
    const Z *hp = H + arow + (int64_t)(kbeg + q) * ldh;
    const int64_t hstep = 4 * ldh;   // one k step = 4 columns of H
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

    // Complex multiply-accumulate of one 4-wide k step on all WN tiles:
    // Re += hr*yr - hi*yi, Im += hr*yi + hi*yr; the two halves of each
    // accumulator are 2*WN instructions apart so dependent MFMAs never
    // issue back to back.
#define CHASE_KSTEP(hv, yv)                                                   \
    {                                                                         \
        const double nhy_ = -(hv).y;                                          \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            cr[c] = mfma64((hv).x, (yv)[c].x, cr[c]);                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            ci[c] = mfma64((hv).x, (yv)[c].y, ci[c]);                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            cr[c] = mfma64(nhy_, (yv)[c].y, cr[c]);                           \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            ci[c] = mfma64((hv).y, (yv)[c].x, ci[c]);                         \
    }

    const int nsteps = (kend - kbeg) >> 2;
    if constexpr (PD == 0) {
        // Wide tiles (MFMA-bound): the operands of step s + 1 load while
        // step s computes; at 4*WN MFMAs per step this covers the latency.
        if (nsteps > 0) {
            Z h = *hp;
            Z y[WN];
#pragma unroll
            for (int c = 0; c < WN; ++c) y[c] = yp[ycol[c]];
            for (int st = 0; st + 1 < nsteps; ++st) {
                const Z *hn_p = hp + (int64_t)(st + 1) * hstep;
                const Z *yn_p = yp + (int64_t)(st + 1) * ystep;
                Z hn = *hn_p;
                Z yn[WN];
#pragma unroll
                for (int c = 0; c < WN; ++c) yn[c] = yn_p[ycol[c]];
                CHASE_KSTEP(h, y);
                h = hn;
#pragma unroll
                for (int c = 0; c < WN; ++c) y[c] = yn[c];
            }
            CHASE_KSTEP(h, y);
        }
    } else {
        // Narrow tiles: a register ring of R = PD + 1 k steps, step t in
        // stage t % R.  Before the MFMAs of step t the operands of step
        // t + PD are loaded into the stage step t - 1 just freed, so each
        // wave keeps PD steps of loads in flight (short steps need many).
        // The steady-state loop has no bounds checks; the remainder does.
        constexpr int R = PD + 1;
        Z hr[R];
        Z yr[R][WN];
#define CHASE_LOAD(stage, step)                                               \
    {                                                                         \
        hr[stage] = hp[(int64_t)(step) * hstep];                              \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            yr[stage][c] = yp[(int64_t)(step) * ystep + ycol[c]];             \
    }
#pragma unroll
        for (int j = 0; j < PD; ++j)
            if (j < nsteps) CHASE_LOAD(j, j);
        int s0 = 0;
        for (; s0 + R + PD <= nsteps; s0 += R) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                CHASE_LOAD((j + PD) % R, s0 + j + PD);
                CHASE_KSTEP(hr[j], yr[j]);
            }
        }
        for (; s0 < nsteps; s0 += R) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int st = s0 + j;
                if (st < nsteps) {
                    if (st + PD < nsteps) CHASE_LOAD((j + PD) % R, st + PD);
                    CHASE_KSTEP(hr[j], yr[j]);
                }
            }
        }
#undef CHASE_LOAD
    }
    const int k = kbeg + 4 * nsteps;
    if (k < kend) {
        // Ragged tail of K: lanes whose k is past the end contribute zero
        // and do not load.
        const bool ok = (k + q) < kend;
        const Z *hq = hp + (int64_t)nsteps * hstep;
        const Z *yq = yp + (int64_t)nsteps * ystep;
        Z h = ok ? *hq : Z{0.0, 0.0};
        Z y[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) y[c] = ok ? yq[ycol[c]] : Z{0.0, 0.0};
        CHASE_KSTEP(h, y);
    }
#undef CHASE_KSTEP

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

// Prefetch depth per tile width (0 = one step ahead, no ring): narrow
// tiles have short k steps and need more loads in flight to cover HBM
// latency; measured on MI355X at N = 24000 the ring helps up to WN = 4 and
// costs registers (and speed) beyond.
constexpr int prefetch_depth(int wn) {
    return wn == 1 ? 8 : wn == 2 ? 6 : wn == 3 ? 4 : wn == 4 ? 2 : 0;
}


template <int WN>
void launch_wn(const FilterPlan &p, const Z *H, int64_t ldh, int N, const Z *Y,
               int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n,
               double a, double b, double g, Z *part, hipStream_t s) {
    const int groups = (p.rb + 7) / 8;
    const int nblocks = groups * 8 * p.cb * p.splits;
    if (p.splits == 1) {
        hipLaunchKernelGGL((k_filter<WN, prefetch_depth(WN), true>), dim3(nblocks), dim3(256), 0, s,
                           H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, p.rb,
                           p.cb, 1, p.kchunk, nullptr);
    } else {
        hipLaunchKernelGGL((k_filter<WN, prefetch_depth(WN), false>), dim3(nblocks), dim3(256), 0,
                           s, H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g,
                           p.rb, p.cb, p.splits, p.kchunk, part);
    }
}


}  // namespace filter_detail
}  // namespace chase
