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

#include "k_filter_kern.h"

#include <algorithm>
#include <vector>

namespace chase {

void launch_filter_wide(const FilterPlan &p, const Z *H, int64_t ldh, int N,
                        const Z *Y, int64_t ldy, const Z *X, int64_t ldx, Z *W,
                        int64_t ldw, int n, double a, double b, double g, Z *part,
                        hipStream_t s);
void launch_filter_group_wide(int wn, const FilterPlan *plans, const FilterCall *calls,
                              int count, hipStream_t s);

namespace {
using namespace filter_detail;

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
        const Z xv = g != 0.0 ? X[row * ldx + col] : Z{0.0, 0.0};
        W[row * ldw + col] = filter_epilogue(sr, si, yv, xv, a, b, g);
    }
}

// The reductions of several split GEMMs in one grid: GEMM i owns blocks
// [start[i], start[i+1]) and strides over its own N*n entries.
struct ReduceGroupArgs {
    int count;
    int start[kMaxGroup + 1];
    FilterArgs p[kMaxGroup];
};

__global__ __launch_bounds__(256) void k_filter_reduce_group(const ReduceGroupArgs G) {
    int i = 0;
    while (i + 1 < G.count && (int)blockIdx.x >= G.start[i + 1]) ++i;
    const FilterArgs &A = G.p[i];
    const int nblk = G.start[i + 1] - G.start[i];
    const int64_t total = (int64_t)A.N * A.n;
    for (int64_t t = (blockIdx.x - G.start[i]) * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)nblk * blockDim.x) {
        const int64_t row = t / A.n;
        const int col = (int)(t - row * A.n);
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < A.splits; ++s) {
            const Z p = A.part[(int64_t)s * total + t];
            sr += p.x;
            si += p.y;
        }
        const Z yv = A.Y[row * A.ldy + col];
        const Z xv = A.g != 0.0 ? A.X[row * A.ldx + col] : Z{0.0, 0.0};
        A.W[row * A.ldw + col] = filter_epilogue(sr, si, yv, xv, A.a, A.b, A.g);
    }
}

int reduce_blocks(int64_t N, int n) {
    return (int)std::min<int64_t>(((int64_t)N * n + 255) / 256, 4096);
}

void filter_group_round(const std::vector<std::pair<FilterCall, FilterPlan>> &rd,
                        hipStream_t s);

}  // namespace

namespace {

// Tile plan for cb column blocks of wn 16-column tiles over N rows.  K
// splits balance the workgroups over the 256 CUs: resident workgroups per
// CU = waves per SIMD of the tile's register budget (hipcc resource usage
// for gfx950); a round of `slots` workgroups runs concurrently, and a
// workgroup's time falls as 1/splits.  Splitting costs a partial-sum pass
// (2 * splits * N * n * 16 bytes), charged at 2% per split.  A split keeps
// at least 512 columns of H, 128 below N = 8192: there the row blocks alone
// fill a third of the CUs or less (N = 2000, 32 row blocks: 3 splits under
// the 512 floor, 7 under 128, and a D + K N = 2000 solve 19.6 -> 15.5 ms;
// 5 or 14 splits were both slower, 17.0 ms).
FilterPlan plan_blocks(int64_t N, int wn, int cb) {
    static const int occ[11] = {0, 3, 2, 2, 2, 3, 2, 2, 2, 1, 1};
    FilterPlan p{};
    p.wn = wn;
    p.cb = cb;
    p.rb = (int)((N + 63) / 64);
    const int64_t slots = 256 * (int64_t)occ[p.wn];
    const int64_t units = (int64_t)p.rb * p.cb;
    double best = 1e300;
    int bests = 1;
    for (int sp = 1; sp <= 16; ++sp) {
        if (sp > 1 && N / sp < (N < 8192 ? 128 : 512)) break;
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

FilterPlan filter_plan(int64_t N, int n) {
    if (n < 1 || n > kMaxTileCols) throw Error(7, "filter_plan: bad column count");
    return plan_blocks(N, (n + 15) / 16, 1);
}

std::vector<FilterPiece> filter_pieces(int64_t N, int n) {
    std::vector<FilterPiece> out;
    if (n <= 0) return out;
    const int tiles = (n + 15) / 16, maxt = kMaxTileCols / 16;
    const int nc = (tiles + maxt - 1) / maxt;
    if (tiles % nc == 0) {
        out.push_back(FilterPiece{0, n, plan_blocks(N, tiles / nc, nc)});
        return out;
    }
    for (const auto &ch : column_chunks(n))
        out.push_back(FilterPiece{ch.first, ch.second, filter_plan(N, ch.second)});
    return out;
}

size_t filter_partial_elems(int64_t N, int n) {
    size_t e = 0;
    for (const FilterPiece &pc : filter_pieces(N, n))
        if (pc.p.splits > 1) e = std::max(e, (size_t)pc.p.splits * (size_t)N * (size_t)pc.n);
    return e;
}

void filter_gemm(const Z *H, int64_t ldh, int64_t N64, const Z *Y, int64_t ldy,
                 const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
                 double b, double g, Z *part, hipStream_t s,
                 hipEvent_t after_mfma) {
    if (n <= 0 || N64 <= 0) return;
    check_buffer_strides(ldh, ldy);
    const int N = (int)N64;
    const auto pieces = filter_pieces(N64, n);
    for (size_t i = 0; i < pieces.size(); ++i) {
        const FilterPlan &p = pieces[i].p;
        const int c0 = pieces[i].c0, nc = pieces[i].n;
        const Z *Yc = Y + c0, *Xc = X ? X + c0 : nullptr;
        Z *Wc = W + c0;
        if (p.splits > 1 && !part) throw Error(7, "filter_gemm: missing partials");
        switch (p.wn) {
#define CASE(w) \
    case w: launch_wn<w>(p, H, ldh, N, Yc, ldy, Xc, ldx, Wc, ldw, nc, a, b, g, part, s); break;
            CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
            case 9:
            case 10:
                launch_filter_wide(p, H, ldh, N, Yc, ldy, Xc, ldx, Wc, ldw, nc, a, b, g, part,
                                   s);
                break;
            default: throw Error(7, "filter_gemm: bad tile width");
        }
        check_launch("k_filter");
        if (after_mfma && i + 1 == pieces.size()) CHASE_HIP(hipEventRecord(after_mfma, s));
        if (p.splits > 1) {
            hipLaunchKernelGGL(k_filter_reduce, dim3(reduce_blocks(N, nc)), dim3(256), 0, s,
                               part, p.splits, N, nc, Yc, ldy, Xc, ldx, Wc, ldw, a, b, g);
            check_launch("k_filter_reduce");
        }
    }
}

void filter_gemm_group(const FilterCall *calls, int count, hipStream_t s) {
    // Round r holds piece r of every call (see filter_pieces), so each
    // call's split-K scratch is used by one piece at a time, in the order
    // filter_gemm uses it.
    std::vector<std::vector<std::pair<FilterCall, FilterPlan>>> rounds;
    for (int i = 0; i < count; ++i) {
        if (calls[i].n <= 0 || calls[i].N <= 0) continue;
        check_buffer_strides(calls[i].ldh, calls[i].ldy);
        const auto pieces = filter_pieces(calls[i].N, calls[i].n);
        if (rounds.size() < pieces.size()) rounds.resize(pieces.size());
        for (size_t r = 0; r < pieces.size(); ++r) {
            FilterCall c = calls[i];
            c.Y += pieces[r].c0;
            if (c.X) c.X += pieces[r].c0;
            c.W += pieces[r].c0;
            c.n = pieces[r].n;
            rounds[r].emplace_back(c, pieces[r].p);
        }
    }
    for (const auto &rd : rounds) filter_group_round(rd, s);
}

namespace {
// One grouped launch per tile width present, then the split GEMMs'
// reductions.
void filter_group_round(const std::vector<std::pair<FilterCall, FilterPlan>> &rd,
                        hipStream_t s) {
    std::vector<FilterPlan> plan;
    std::vector<FilterCall> live;
    for (const auto &cp : rd) {
        if (cp.second.splits > 1 && !cp.first.part)
            throw Error(7, "filter_gemm_group: missing partials");
        live.push_back(cp.first);
        plan.push_back(cp.second);
    }
    // MFMA launches, one per tile width present (chunks of kMaxGroup).
    for (int wn = 1; wn <= 10; ++wn) {
        std::vector<FilterPlan> pw;
        std::vector<FilterCall> cw;
        for (size_t i = 0; i < live.size(); ++i)
            if (plan[i].wn == wn) {
                pw.push_back(plan[i]);
                cw.push_back(live[i]);
            }
        for (size_t c0 = 0; c0 < pw.size(); c0 += kMaxGroup) {
            const int m = (int)std::min<size_t>(kMaxGroup, pw.size() - c0);
            switch (wn) {
#define CASE(w) \
    case w: launch_group_wn<w>(pw.data() + c0, cw.data() + c0, m, s); break;
                CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
                default: launch_filter_group_wide(wn, pw.data() + c0, cw.data() + c0, m, s);
            }
            check_launch("k_filter_group");
        }
    }
    // The split GEMMs' ordered reductions, in one grid per kMaxGroup.
    std::vector<size_t> split;
    for (size_t i = 0; i < live.size(); ++i)
        if (plan[i].splits > 1) split.push_back(i);
    for (size_t c0 = 0; c0 < split.size(); c0 += kMaxGroup) {
        const int m = (int)std::min<size_t>(kMaxGroup, split.size() - c0);
        ReduceGroupArgs G{};
        G.count = m;
        int off = 0;
        for (int j = 0; j < m; ++j) {
            const size_t i = split[c0 + j];
            G.start[j] = off;
            G.p[j] = filter_args(plan[i], live[i]);
            off += reduce_blocks(live[i].N, live[i].n);
        }
        G.start[m] = off;
        hipLaunchKernelGGL(k_filter_reduce_group, dim3(off), dim3(256), 0, s, G);
        check_launch("k_filter_reduce_group");
    }
}

}  // namespace

}  // namespace chase
