// Column plan of the filter GEMMs (both precisions): how a block of n
// columns is cut into launches and how each launch is tiled.  Shared by the
// launchers and the partial-sum sizing; a filter kernel's measured profile
// depends on it (with the kernel sources).
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace chase {

struct FilterPlan {
    int wn;       // 16-column blocks per wave (1..10)
    int cb;       // column blocks of 16*wn columns
    int rb;       // row blocks of 64 rows
    int splits;   // K splits (1 = epilogue fused)
    int kchunk;   // K rows per split (multiple of 4)
};
// Tile plan of one GEMM of at most kMaxTileCols columns.
constexpr int kMaxTileCols = 160;   // 10 tiles of 16 columns per wave
FilterPlan filter_plan(int64_t N, int n);
// Wider blocks run as balanced chunks of whole 16-column tiles, each its
// own GEMM (at most kMaxTileCols columns), so only the last 16-column tile
// of the block carries padding.  Returns (first column, columns) pairs.
inline std::vector<std::pair<int, int>> column_chunks(int n) {
    std::vector<std::pair<int, int>> out;
    if (n <= 0) return out;
    const int tiles = (n + 15) / 16;
    const int maxt = kMaxTileCols / 16;
    const int nc = (tiles + maxt - 1) / maxt;
    int t0 = 0;
    for (int i = 0; i < nc; ++i) {
        const int w = tiles / nc + (i < tiles % nc ? 1 : 0);
        const int c0 = 16 * t0, c1 = std::min(n, 16 * (t0 + w));
        out.emplace_back(c0, c1 - c0);
        t0 += w;
    }
    return out;
}
// The launches of a filter GEMM of n columns, in order: one launch when
// the columns fit one tile block or split evenly into blocks of equal
// width (several column blocks in one grid), otherwise one launch per
// balanced chunk.  Columns [c0, c0 + n) with tile plan p.
struct FilterPiece {
    int c0, n;
    FilterPlan p;
};
std::vector<FilterPiece> filter_pieces(int64_t N, int n);
// Split-K scratch (elements) for a filter GEMM of n columns: the largest
// piece's need, pieces running one after another.
size_t filter_partial_elems(int64_t N, int n);

// The same for the FP32 filter (its own register budgets, so its own split
// counts); partials in complex64 elements.
FilterPlan filter32_plan(int64_t N, int n);
std::vector<FilterPiece> filter32_pieces(int64_t N, int n);
size_t filter32_partial_elems(int64_t N, int n);

}  // namespace chase
