// FP32 Chebyshev filter step for the mixed-precision form:
//     W = a * Hc Y + b * Y + g * X
// with Hc the complex64 shadow of H (column-major) and Y, X, W complex64
// row-major blocks, FP32 MFMA (v_mfma_f32_16x16x4_f32) and FP32
// accumulation.  Same tiling and ordering as the FP64 kernel (k_filter_kern.h)
// with 8-byte operands; the FP32 MFMA issues twice as often, so narrow tiles
// keep deeper prefetch rings.  Also the FP64 <-> FP32 conversion kernels for
// the shadow and the vector blocks.
#include "common.h"

#include <algorithm>

namespace chase {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma32(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// H steps in flight and Y buffers per FP32 tile width (measured on MI355X
// at N = 24000 against 8 and 2: 16 and 4 are 2-4% faster at widths 5-9;
// the full-operand ring of 4-6 steps they replaced was 8-32% slower).  The
// narrow tiles carry Y as far ahead as H.
constexpr int h_ring32(int wn) { return wn >= 5 ? 16 : wn >= 3 ? 12 : 16; }
constexpr int y_bufs32(int wn) { return wn >= 5 ? 4 : h_ring32(wn); }
constexpr int kHRing32Max = 16;

// Raw buffer over `bytes` bytes at `base` (loads past them return zero),
// and one 8-byte load from it at a per-lane and a scalar byte offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc32(const void *base, int64_t bytes) {
    const int num = (int)(bytes <= 0 ? 0 : bytes < 0x7fffffff ? bytes : 0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, num, 0x00020000);
}
__device__ __forceinline__ C buffer_load_c(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __builtin_bit_cast(C, v);
}

template <int WN, int PD, bool FUSED>
__global__ __launch_bounds__(256) void k_filter32(
    const C *__restrict__ H, int64_t ldh, int N, const C *__restrict__ Y,
    int64_t ldy, const C *X, int64_t ldx, C *W, int64_t ldw, int n, float a,
    float b, float g, int rb_count, int cb_count, int splits, int kchunk,
    C *__restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform buffer bases
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
    const int arow = min(row0 + r, N - 1);
    const C *hp = H + arow + (int64_t)(kbeg + q) * ldh;
    const int64_t hstep = 4 * ldh;
    int ycol[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) ycol[c] = min(col0 + 16 * c + r, n - 1);
    const C *yp = Y + (int64_t)(kbeg + q) * ldy;
    const int64_t ystep = 4 * ldy;
    v4f cr[WN], ci[WN];
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        cr[c] = v4f{0.f, 0.f, 0.f, 0.f};
        ci[c] = v4f{0.f, 0.f, 0.f, 0.f};
    }
#define CHASE_KSTEP32(hv, yv)                                                 \
    {                                                                         \
        const float nhy_ = -(hv).y;                                           \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            cr[c] = mfma32((hv).x, (yv)[c].x, cr[c]);                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            ci[c] = mfma32((hv).x, (yv)[c].y, ci[c]);                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            cr[c] = mfma32(nhy_, (yv)[c].y, cr[c]);                           \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            ci[c] = mfma32((hv).y, (yv)[c].x, ci[c]);                         \
    }
    const int nsteps = (kend - kbeg) >> 2;
    {
        // A ring of DH steps of H loads in flight and Y loaded YB - 1 steps
        // ahead into YB buffers (step t uses H stage t % DH and Y buffer
        // t % YB), through raw buffer loads whose base moves once per ring
        // turn and covers only the steps left, so loads past the end return
        // zero and the loop needs no guards (the FP64 kernel's scheme, with
        // more steps in flight: an FP32 MFMA takes half as long).
        constexpr int DH = h_ring32(WN), YB = y_bufs32(WN);
        static_assert(DH % YB == 0, "the Y buffer follows the H stage");
        const char *hbase = reinterpret_cast<const char *>(H + row0 + (int64_t)kbeg * ldh);
        const char *ybase = reinterpret_cast<const char *>(Y + (int64_t)kbeg * ldy);
        const int hs = (int)(4 * ldh * (int64_t)sizeof(C));
        const int ys = (int)(4 * ldy * (int64_t)sizeof(C));
        const int hvo = (int)((arow - row0 + (int64_t)q * ldh) * sizeof(C));
        int yvo[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) yvo[c] = (int)(((int64_t)q * ldy + ycol[c]) * sizeof(C));
        C hr[DH];
        C yb[YB][WN];
        auto h_rsrc = [&](int st) {
            return buffer_rsrc32(hbase + (int64_t)st * hs, (int64_t)(nsteps - st) * hs);
        };
        auto y_rsrc = [&](int st) {
            return buffer_rsrc32(ybase + (int64_t)st * ys, (int64_t)(nsteps - st) * ys);
        };
        __amdgpu_buffer_rsrc_t rh = h_rsrc(0), ry = y_rsrc(0);
#define CHASE_LOADH32(stage, rel) hr[stage] = buffer_load_c(rh, hvo, (rel) * hs);
#define CHASE_LOADY32(buf, rel)                                               \
    {                                                                         \
        _Pragma("unroll") for (int c = 0; c < WN; ++c)                        \
            yb[buf][c] = buffer_load_c(ry, yvo[c], (rel) * ys);               \
    }
        if (nsteps > 0) {
#pragma unroll
            for (int j = 0; j < DH; ++j) CHASE_LOADH32(j, j);
#pragma unroll
            for (int j = 0; j < YB - 1; ++j) CHASE_LOADY32(j, j);
        }
        for (int s0 = 0; s0 < nsteps; s0 += DH) {
            // rh and ry are based at step s0.
#pragma unroll
            for (int j = 0; j < DH; ++j) {
                CHASE_LOADY32((j + YB - 1) % YB, j + YB - 1);
                // (the loads stay ahead of the step's MFMAs: left alone the
                // scheduler sinks them next to their use)
                __builtin_amdgcn_sched_barrier(0);
                CHASE_KSTEP32(hr[j], yb[j % YB]);
                CHASE_LOADH32(j, j + DH);
            }
            rh = h_rsrc(s0 + DH);
            ry = y_rsrc(s0 + DH);
        }
#undef CHASE_LOADH32
#undef CHASE_LOADY32
    }
    const int k = kbeg + 4 * nsteps;
    if (k < kend) {
        const bool ok = (k + q) < kend;
        const C *hq = hp + (int64_t)nsteps * hstep;
        const C *yq = yp + (int64_t)nsteps * ystep;
        C h = ok ? *hq : C{0.f, 0.f};
        C y[WN];
#pragma unroll
        for (int c = 0; c < WN; ++c) y[c] = ok ? yq[ycol[c]] : C{0.f, 0.f};
        CHASE_KSTEP32(h, y);
    }
#undef CHASE_KSTEP32
    // Accumulator layout of the 16x16x4 FP32 MFMA: register v of lane (r, q)
    // holds row 4q + v of column r.
#pragma unroll
    for (int c = 0; c < WN; ++c) {
        const int col = col0 + 16 * c + r;
        if (col >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + 4 * q + v;
            if (row >= N) continue;
            const float sr = cr[c][v], si = ci[c][v];
            if (FUSED) {
                const C yv = Y[(int64_t)row * ldy + col];
                C o;
                o.x = a * sr + b * yv.x;
                o.y = a * si + b * yv.y;
                if (g != 0.f) {
                    const C xv = X[(int64_t)row * ldx + col];
                    o.x += g * xv.x;
                    o.y += g * xv.y;
                }
                W[(int64_t)row * ldw + col] = o;
            } else {
                part[((int64_t)sp * N + row) * n + col] = C{sr, si};
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_filter32_reduce(
    const C *__restrict__ part, int splits, int N, int n, const C *Y,
    int64_t ldy, const C *X, int64_t ldx, C *W, int64_t ldw, float a, float b,
    float g) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / n;
        const int col = (int)(t - row * n);
        float sr = 0.f, si = 0.f;
        for (int s = 0; s < splits; ++s) {
            const C p = part[(int64_t)s * total + t];
            sr += p.x;
            si += p.y;
        }
        const C yv = Y[row * ldy + col];
        C o;
        o.x = a * sr + b * yv.x;
        o.y = a * si + b * yv.y;
        if (g != 0.f) {
            const C xv = X[row * ldx + col];
            o.x += g * xv.x;
            o.y += g * xv.y;
        }
        W[row * ldw + col] = o;
    }
}

// The kernels' PD template argument: the H ring of the width.
constexpr int prefetch_depth32(int wn) { return h_ring32(wn); }

template <int WN>
void launch32(const FilterPlan &p, const C *H, int64_t ldh, int N, const C *Y,
              int64_t ldy, const C *X, int64_t ldx, C *W, int64_t ldw, int n,
              float a, float b, float g, C *part, hipStream_t s) {
    const int groups = (p.rb + 7) / 8;
    const int nblocks = groups * 8 * p.cb * p.splits;
    if (p.splits == 1)
        hipLaunchKernelGGL((k_filter32<WN, prefetch_depth32(WN), true>), dim3(nblocks),
                           dim3(256), 0, s, H, ldh, N, Y, ldy, X, ldx, W, ldw, n,
                           a, b, g, p.rb, p.cb, 1, p.kchunk, nullptr);
    else
        hipLaunchKernelGGL((k_filter32<WN, prefetch_depth32(WN), false>),
                           dim3(nblocks), dim3(256), 0, s, H, ldh, N, Y, ldy, X,
                           ldx, W, ldw, n, a, b, g, p.rb, p.cb, p.splits,
                           p.kchunk, part);
}

// ------------------------------------------------------------ conversions
__global__ void k_z2c_mat(const Z *__restrict__ H, int64_t ldh, C *__restrict__ Hc,
                          int64_t ldc, int64_t N) {
    const int64_t total = N * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / N, i = t - j * N;
        const Z v = H[i + j * ldh];
        Hc[i + j * ldc] = C{(float)v.x, (float)v.y};
    }
}

__global__ void k_z2c_blk(const Z *__restrict__ V, int64_t ldv, C *__restrict__ Vc,
                          int64_t ldc, int N, int n) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        const Z v = V[i * ldv + j];
        Vc[i * ldc + j] = C{(float)v.x, (float)v.y};
    }
}

__global__ void k_c2z_blk(const C *__restrict__ Vc, int64_t ldc, Z *__restrict__ V,
                          int64_t ldv, int N, int n) {
    const int64_t total = (int64_t)N * n;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / n, j = t - i * n;
        const C v = Vc[i * ldc + j];
        V[i * ldv + j] = Z{(double)v.x, (double)v.y};
    }
}

inline int grid_for(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384));
}

}  // namespace

namespace {

// As the FP64 plan, with the FP32 kernels' register budgets.
FilterPlan plan32_blocks(int64_t N, int wn, int cb) {
    static const int occ[11] = {0, 4, 3, 2, 2, 2, 1, 1, 1, 1, 1};
    FilterPlan p{};
    p.wn = wn;
    p.cb = cb;
    p.rb = (int)((N + 63) / 64);
    const int64_t slots = 256 * (int64_t)occ[p.wn];
    const int64_t units = (int64_t)p.rb * p.cb;
    double best = 1e300;
    int bests = 1;
    for (int sp = 1; sp <= 16; ++sp) {
        if (sp > 1 && N / sp < 512) break;
        const double rounds = (double)((units * sp + slots - 1) / slots);
        const double cost = rounds / sp + 0.02 * (sp - 1);
        if (cost < best - 1e-12) {
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

}  // namespace

FilterPlan filter32_plan(int64_t N, int n) {
    if (n < 1 || n > kMaxTileCols) throw Error(7, "filter32_plan: bad column count");
    return plan32_blocks(N, (n + 15) / 16, 1);
}

std::vector<FilterPiece> filter32_pieces(int64_t N, int n) {
    std::vector<FilterPiece> out;
    if (n <= 0) return out;
    const int tiles = (n + 15) / 16, maxt = kMaxTileCols / 16;
    const int nc = (tiles + maxt - 1) / maxt;
    if (tiles % nc == 0) {
        out.push_back(FilterPiece{0, n, plan32_blocks(N, tiles / nc, nc)});
        return out;
    }
    for (const auto &ch : column_chunks(n))
        out.push_back(FilterPiece{ch.first, ch.second, filter32_plan(N, ch.second)});
    return out;
}

size_t filter32_partial_elems(int64_t N, int n) {
    size_t e = 0;
    for (const FilterPiece &pc : filter32_pieces(N, n))
        if (pc.p.splits > 1) e = std::max(e, (size_t)pc.p.splits * (size_t)N * (size_t)pc.n);
    return e;
}

void filter32_gemm(const C *H, int64_t ldh, int64_t N64, const C *Y, int64_t ldy,
                   const C *X, int64_t ldx, C *W, int64_t ldw, int n, float a,
                   float b, float g, C *part, hipStream_t s, hipEvent_t after_mfma) {
    if (n <= 0 || N64 <= 0) return;
    {
        // 32-bit buffer offsets of up to 2 h_ring32 k steps (wide tiles)
        const int64_t lim = ((int64_t)1 << 31) / (2 * kHRing32Max * 4 * (int64_t)sizeof(C));
        if (ldh >= lim || ldy >= lim)
            throw Error(1, "filter: leading dimension too large for 32-bit buffer offsets");
    }
    const int N = (int)N64;
    const auto pieces = filter32_pieces(N64, n);
    for (size_t i = 0; i < pieces.size(); ++i) {
        const FilterPlan &p = pieces[i].p;
        const int c0 = pieces[i].c0, nc = pieces[i].n;
        const C *Yc = Y + c0, *Xc = X ? X + c0 : nullptr;
        C *Wc = W + c0;
        if (p.splits > 1 && !part) throw Error(7, "filter32_gemm: missing partials");
        switch (p.wn) {
#define CASE(w) case w: launch32<w>(p, H, ldh, N, Yc, ldy, Xc, ldx, Wc, ldw, nc, a, b, g, part, s); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
            default: throw Error(7, "filter32_gemm: bad tile width");
        }
        check_launch("k_filter32");
        if (after_mfma && i + 1 == pieces.size()) CHASE_HIP(hipEventRecord(after_mfma, s));
        if (p.splits > 1) {
            const int64_t total = (int64_t)N * nc;
            hipLaunchKernelGGL(k_filter32_reduce,
                               dim3((int)std::min<int64_t>((total + 255) / 256, 4096)),
                               dim3(256), 0, s, part, p.splits, N, nc, Yc, ldy, Xc, ldx, Wc,
                               ldw, a, b, g);
            check_launch("k_filter32_reduce");
        }
    }
}

void z2c_matrix(const Z *H, int64_t ldh, C *Hc, int64_t ldc, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_z2c_mat, dim3(grid_for(N * N)), dim3(256), 0, s, H, ldh, Hc,
                       ldc, N);
    check_launch("k_z2c_mat");
}

void z2c_block(const Z *V, int64_t ldv, C *Vc, int64_t ldc, int64_t N, int n,
               hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_z2c_blk, dim3(grid_for(N * n)), dim3(256), 0, s, V, ldv, Vc,
                       ldc, (int)N, n);
    check_launch("k_z2c_blk");
}

void c2z_block(const C *Vc, int64_t ldc, Z *V, int64_t ldv, int64_t N, int n,
               hipStream_t s) {
    if (N <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_c2z_blk, dim3(grid_for(N * n)), dim3(256), 0, s, Vc, ldc, V,
                       ldv, (int)N, n);
    check_launch("k_c2z_blk");
}

}  // namespace chase
