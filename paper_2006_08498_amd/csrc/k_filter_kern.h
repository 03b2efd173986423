// Filter GEMM kernel template, shared by the two translation units that
// instantiate it (k_filter.hip: tile widths 1-8; k_filter_wide.hip: widths
// 9-10; both built with the VGPR form of MFMA, in which the register
// allocator keeps every width's accumulators in place through the k loop).
#pragma once

#include "common.h"

namespace chase {
namespace filter_detail {


typedef double v4d __attribute__((ext_vector_type(4)));

// W = a * (H Y) + b * Y + g * X for one entry, with every rounding spelled
// out (explicit fused multiply-adds), so the direct, split and grouped
// launches give bitwise the same value whatever the compiler contracts.
__device__ __forceinline__ Z filter_epilogue(double sr, double si, Z yv, Z xv, double a,
                                             double b, double g) {
    Z o;
    o.x = __builtin_fma(a, sr, b * yv.x);
    o.y = __builtin_fma(a, si, b * yv.y);
    o.x = __builtin_fma(g, xv.x, o.x);
    o.y = __builtin_fma(g, xv.y, o.y);
    return o;
}

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Arguments of one filter GEMM as the kernels see them.
struct FilterArgs {
    const Z *H;
    int64_t ldh;
    const Z *Y;
    int64_t ldy;
    const Z *X;
    int64_t ldx;
    Z *W;
    int64_t ldw;
    Z *part;
    double a, b, g;
    int N, n, rb_count, cb_count, splits, kchunk;
};

// Up to this many GEMMs share one grouped launch (the arguments travel as
// kernel arguments, about 2 KB).
constexpr int kMaxGroup = 16;
struct FilterGroupArgs {
    int count;
    int start[kMaxGroup + 1];   // first workgroup of each GEMM (multiples of 8)
    FilterArgs p[kMaxGroup];
};

// Raw buffer over `bytes` bytes at `base` (loads past them return zero),
// and one 16-byte load from it at a per-lane and a scalar byte offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, int64_t bytes) {
    const int num = (int)(bytes <= 0 ? 0 : bytes < 0x7fffffff ? bytes : 0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, num, 0x00020000);
}
__device__ __forceinline__ Z buffer_load_z(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return __builtin_bit_cast(Z, v);
}
// The same load marked non-temporal (cache policy nt): H is streamed once
// per launch, and the hint keeps it from displacing the Y block, which every
// row panel re-reads, in L2 (1-3% faster at every tile width at N = 24000;
// the FP32 kernel gained nothing from it).
__device__ __forceinline__ Z buffer_load_z_stream(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    constexpr int kNonTemporal = 2;
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kNonTemporal);
    return __builtin_bit_cast(Z, v);
}

// Ring of each tile width: H steps in flight (the kernels' PD) and Y
// buffers.  Measured on MI355X at N = 24000: 8 H steps against 4 are 1.8%
// faster at 9 tiles, 6 are best at 5-8; the narrow tiles carry Y as far
// ahead as H (2-5% faster at widths 1-4 than the full-operand rings of 9,
// 7, 5 and 3 steps with 64-bit addresses they replaced).
constexpr int h_ring(int wn) { return wn >= 9 ? 8 : wn >= 4 ? 6 : wn == 3 ? 8 : wn == 2 ? 12 : 16; }
constexpr int y_bufs(int wn) { return wn >= 5 ? 2 : h_ring(wn); }
constexpr int kHRingMax = 16;

// Workgroup `id` of one GEMM's grid: a 64-row block of H times a block of
// 16*WN columns over one K range.
template <int WN, int PD, bool FUSED>
__device__ __forceinline__ void filter_tile(
    const Z *__restrict__ H, int64_t ldh, int N, const Z *__restrict__ Y,
    int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
    double b, double g, int rb_count, int cb_count, int splits, int kchunk,
    Z *__restrict__ part, int id) {
    const int lane = threadIdx.x & 63;
    // (readfirstlane: the compiler then knows the wave index, and the buffer
    // bases below, are uniform across the wave)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;

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
    {
        // A ring of PD steps of H loads in flight and Y loaded YB - 1 steps
        // ahead into YB buffers (step t uses H stage t % PD and Y buffer
        // t % YB).  H streams from HBM; Y comes mostly from L2, so the wide
        // (MFMA-bound) tiles load it one step ahead, and the narrow ones,
        // whose k steps are short, as far ahead as H.  The loads are buffer
        // loads: a per-lane 32-bit offset plus a scalar offset from a base
        // that moves once per ring turn, so a step costs no 64-bit address
        // registers (which the accumulators of the widest tiles need), and
        // each buffer covers only the steps left, so loads past the end
        // return zeros (hardware range check) and the loop needs no guards
        // (a guarded load makes the compiler wait for every load in flight;
        // the extra steps add nothing).
        constexpr int DH = PD, YB = y_bufs(WN);
        static_assert(DH % YB == 0, "the Y buffer follows the H stage");
        const char *hbase = reinterpret_cast<const char *>(H + row0 + (int64_t)kbeg * ldh);
        const char *ybase = reinterpret_cast<const char *>(Y + (int64_t)kbeg * ldy);
        const int hs = (int)(4 * ldh * (int64_t)sizeof(Z));   // bytes per k step
        const int ys = (int)(4 * ldy * (int64_t)sizeof(Z));
        const int hvo = (int)((arow - row0 + (int64_t)q * ldh) * sizeof(Z));
        int yvo[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) yvo[c] = (int)(((int64_t)q * ldy + ycol[c]) * sizeof(Z));
        Z hr[DH];
        Z yb[YB][WN];
        auto h_rsrc = [&](int st) {
            return buffer_rsrc(hbase + (int64_t)st * hs, (int64_t)(nsteps - st) * hs);
        };
        auto y_rsrc = [&](int st) {
            return buffer_rsrc(ybase + (int64_t)st * ys, (int64_t)(nsteps - st) * ys);
        };
        __amdgpu_buffer_rsrc_t rh = h_rsrc(0), ry = y_rsrc(0);
#define CHASE_LOADH(stage, rel) hr[stage] = buffer_load_z_stream(rh, hvo, (rel) * hs);
#define CHASE_LOADY(buf, rel)                                                 \
    {                                                                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            yb[buf][c] = buffer_load_z(ry, yvo[c], (rel) * ys);               \
    }
        if (nsteps > 0) {
#pragma unroll
            for (int j = 0; j < DH; ++j) CHASE_LOADH(j, j);
#pragma unroll
            for (int j = 0; j < YB - 1; ++j) CHASE_LOADY(j, j);
        }
        for (int s0 = 0; s0 < nsteps; s0 += DH) {
            // rh and ry are based at step s0.
#pragma unroll
            for (int j = 0; j < DH; ++j) {
                CHASE_LOADY((j + YB - 1) % YB, j + YB - 1);
                // (the loads stay ahead of the step's MFMAs: left alone the
                // scheduler sinks them next to their use)
                __builtin_amdgcn_sched_barrier(0);
                CHASE_KSTEP(hr[j], yb[j % YB]);
                CHASE_LOADH(j, j + DH);
            }
            rh = h_rsrc(s0 + DH);
            ry = y_rsrc(s0 + DH);
        }
#undef CHASE_LOADH
#undef CHASE_LOADY
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
                const Z xv = g != 0.0 ? X[(int64_t)row * ldx + col] : Z{0.0, 0.0};
                W[(int64_t)row * ldw + col] = filter_epilogue(sr, si, yv, xv, a, b, g);
            } else {
                part[((int64_t)sp * N + row) * n + col] = Z{sr, si};
            }
        }
    }
}

template <int WN, int PD, bool FUSED>
__global__ __launch_bounds__(256) void k_filter(
    const Z *__restrict__ H, int64_t ldh, int N, const Z *__restrict__ Y,
    int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
    double b, double g, int rb_count, int cb_count, int splits, int kchunk,
    Z *__restrict__ part) {
    filter_tile<WN, PD, FUSED>(H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, rb_count,
                               cb_count, splits, kchunk, part, blockIdx.x);
}

// Several GEMMs of the same tile width in one grid.  Each GEMM's
// workgroups are a contiguous range starting at a multiple of 8, so a
// workgroup lands on the same XCD as in a launch of its own.
template <int WN, int PD>
__global__ __launch_bounds__(256) void k_filter_group(const FilterGroupArgs G) {
    const int id = blockIdx.x;
    int i = 0;
    while (i + 1 < G.count && id >= G.start[i + 1]) ++i;
    const FilterArgs &A = G.p[i];
    const int lid = id - G.start[i];
    if (A.splits == 1)
        filter_tile<WN, PD, true>(A.H, A.ldh, A.N, A.Y, A.ldy, A.X, A.ldx, A.W, A.ldw, A.n,
                                  A.a, A.b, A.g, A.rb_count, A.cb_count, 1, A.kchunk,
                                  nullptr, lid);
    else
        filter_tile<WN, PD, false>(A.H, A.ldh, A.N, A.Y, A.ldy, A.X, A.ldx, A.W, A.ldw, A.n,
                                   A.a, A.b, A.g, A.rb_count, A.cb_count, A.splits,
                                   A.kchunk, A.part, lid);
}

// The kernels' PD: the H ring of the width.
constexpr int prefetch_depth(int wn) { return h_ring(wn); }

// The kernels address H and Y with 32-bit buffer offsets of up to
// 2 h_ring(WN) k steps (4 columns of H, 4 rows of Y each).
inline void check_buffer_strides(int64_t ldh, int64_t ldy) {
    const int64_t lim = ((int64_t)1 << 31) / (2 * kHRingMax * 4 * (int64_t)sizeof(Z));
    if (ldh >= lim || ldy >= lim)
        throw Error(1, "filter: leading dimension too large for 32-bit buffer offsets");
}

inline int filter_blocks(const FilterPlan &p) {
    return (p.rb + 7) / 8 * 8 * p.cb * p.splits;
}

inline FilterArgs filter_args(const FilterPlan &p, const FilterCall &c) {
    FilterArgs A;
    A.H = c.H;
    A.ldh = c.ldh;
    A.Y = c.Y;
    A.ldy = c.ldy;
    A.X = c.X;
    A.ldx = c.ldx;
    A.W = c.W;
    A.ldw = c.ldw;
    A.part = p.splits > 1 ? c.part : nullptr;
    A.a = c.a;
    A.b = c.b;
    A.g = c.g;
    A.N = (int)c.N;
    A.n = c.n;
    A.rb_count = p.rb;
    A.cb_count = p.cb;
    A.splits = p.splits;
    A.kchunk = p.kchunk;
    return A;
}

// One grouped launch of tile width WN (all plans[i].wn == WN).
template <int WN>
void launch_group_wn(const FilterPlan *plans, const FilterCall *calls, int count,
                     hipStream_t s) {
    FilterGroupArgs G{};
    G.count = count;
    int off = 0;
    for (int i = 0; i < count; ++i) {
        G.start[i] = off;
        G.p[i] = filter_args(plans[i], calls[i]);
        off += filter_blocks(plans[i]);
    }
    G.start[count] = off;
    hipLaunchKernelGGL((k_filter_group<WN, prefetch_depth(WN)>), dim3(off), dim3(256), 0, s, G);
}

template <int WN>
void launch_wn(const FilterPlan &p, const Z *H, int64_t ldh, int N, const Z *Y,
               int64_t ldy, const Z *X, int64_t ldx, Z *W, int64_t ldw, int n,
               double a, double b, double g, Z *part, hipStream_t s) {
    const int nblocks = filter_blocks(p);
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
