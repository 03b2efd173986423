// Ingesting H: row stripes of the lower triangle into the column-major
// Hermitian matrix the solver reads, and in-place completion of H from one
// stored triangle.
//
// The paper's reader has each rank read its stripe of rows of the lower half
// and then fills the upper half from the ranks holding the transposed parts
// (Sec. "Matrix generation and the I/O challenge"; the I/O timings are in the
// strong-scaling table of Sec. "Strong scaling").  On one GPU the
// exchange is a transpose through LDS: every stripe is written to both
// triangles as it arrives, so once the stripes cover rows 0..N-1 the matrix
// is complete, Hermitian to the last bit, with a real diagonal.  Both kernels
// move each element once in and (at most) twice out; they are bound by HBM.
#include "common.h"

namespace chase {
namespace {

constexpr int kT = 32;          // tile edge
constexpr int kRowsPerPass = 8; // 256 threads: 32 lanes across, 8 rows down

// Rows [r0, r0 + nrows) of the lower triangle, row-major in `rows` (row r at
// rows + (r - r0) * ldr, columns 0..r read).  Block (bx, by) takes the tile
// of stripe rows by*32.. and columns bx*32..; tiles wholly above the
// diagonal exit at once.
__global__ __launch_bounds__(256) void k_ingest_rows(Z *__restrict__ H, int64_t ldh,
                                                      const Z *__restrict__ rows, int64_t ldr,
                                                      int64_t r0, int64_t nrows) {
    __shared__ Z tile[kT][kT + 1];
    const int tx = threadIdx.x & (kT - 1);
    const int ty = threadIdx.x >> 5;
    const int64_t rt = r0 + (int64_t)blockIdx.y * kT;   // first row of the tile
    const int64_t ct = (int64_t)blockIdx.x * kT;        // first column
    const int64_t rend = r0 + nrows;
    if (ct > rt + kT - 1 || ct >= rend) return;          // above the diagonal
    // Read along the rows (coalesced), write the conjugate into column r of
    // the upper triangle (also along c) and the diagonal; keep the tile.
#pragma unroll
    for (int q = 0; q < kT / kRowsPerPass; ++q) {
        const int rl = ty + kRowsPerPass * q;
        const int64_t r = rt + rl, c = ct + tx;
        if (r < rend && c <= r) {
            const Z v = rows[(r - r0) * ldr + c];
            tile[rl][tx] = v;
            if (c < r) H[c + r * ldh] = make_double2(v.x, -v.y);
            else H[r + r * ldh] = make_double2(v.x, 0.0);
        }
    }
    __syncthreads();
    // Lower triangle: column c of H, rows along the lanes.
#pragma unroll
    for (int q = 0; q < kT / kRowsPerPass; ++q) {
        const int cl = ty + kRowsPerPass * q;
        const int64_t r = rt + tx, c = ct + cl;
        if (r < rend && c < r) H[r + c * ldh] = tile[tx][cl];
    }
}

// In-place completion: block k of the triangular grid takes the tile pair
// (I, J), I >= J.  The source tile holds elements of the stored triangle
// (rows a*32.., columns b*32..), the destination its conjugate transpose
// (rows b*32.., columns a*32..): (a, b) = (I, J) when the lower triangle is
// stored, (J, I) when the upper one is.  Diagonal tiles read their stored
// half before the barrier and write the other half and the (real) diagonal
// after it; no other block touches them.
__global__ __launch_bounds__(256) void k_herm_complete(Z *__restrict__ H, int64_t ldh,
                                                        int64_t N, int lower) {
    __shared__ Z tile[kT][kT + 1];
    const int tx = threadIdx.x & (kT - 1);
    const int ty = threadIdx.x >> 5;
    const int64_t k = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > k) --I;
    while ((I + 1) * (I + 2) / 2 <= k) ++I;
    const int64_t J = k - I * (I + 1) / 2;
    const int64_t a = lower ? I : J, b = lower ? J : I;
    const int64_t ra = a * kT, cb = b * kT;
    // A stored element (row i, column j) qualifies when i > j (lower) or
    // i < j (upper); the diagonal is read too.
    auto stored = [&](int64_t i, int64_t j) { return lower ? i >= j : i <= j; };
#pragma unroll
    for (int q = 0; q < kT / kRowsPerPass; ++q) {
        const int cl = ty + kRowsPerPass * q;
        const int64_t i = ra + tx, j = cb + cl;
        if (i < N && j < N && stored(i, j)) tile[cl][tx] = H[i + j * ldh];
    }
    __syncthreads();
    // Destination (row b*32 + tx, column a*32 + cl) = conj(source (row
    // a*32 + cl, column b*32 + tx)) = conj(tile[tx][cl]).
#pragma unroll
    for (int q = 0; q < kT / kRowsPerPass; ++q) {
        const int cl = ty + kRowsPerPass * q;
        const int64_t si = ra + cl, sj = cb + tx;   // source element
        if (si < N && sj < N && stored(si, sj)) {
            const Z v = tile[tx][cl];
            if (si == sj) H[si + si * ldh] = make_double2(v.x, 0.0);
            else H[sj + si * ldh] = make_double2(v.x, -v.y);
        }
    }
}

}  // namespace

void ingest_rows(Z *H, int64_t ldh, const Z *rows, int64_t ldr, int64_t r0, int64_t nrows,
                 hipStream_t s) {
    if (nrows <= 0) return;
    const dim3 grid((unsigned)((r0 + nrows + kT - 1) / kT), (unsigned)((nrows + kT - 1) / kT));
    hipLaunchKernelGGL(k_ingest_rows, grid, dim3(256), 0, s, H, ldh, rows, ldr, r0, nrows);
    check_launch("k_ingest_rows");
}

void hermitian_complete(Z *H, int64_t ldh, int64_t N, bool lower, hipStream_t s) {
    if (N <= 0) return;
    const int64_t nt = (N + kT - 1) / kT;
    const int64_t blocks = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_herm_complete, dim3((unsigned)blocks), dim3(256), 0, s, H, ldh, N,
                       lower ? 1 : 0);
    check_launch("k_herm_complete");
}

namespace {

// Streams, events and staging buffers of one host ingestion; the destructor
// waits for both streams before anything is released, so an error part-way
// never leaves a copy running into freed memory.
struct HostIngest {
    hipStream_t copy = nullptr;
    hipEvent_t ready[2] = {nullptr, nullptr}, free_[2] = {nullptr, nullptr};
    void *stage[2] = {nullptr, nullptr};
    hipStream_t s;
    explicit HostIngest(hipStream_t st) : s(st) {}
    ~HostIngest() {
        if (copy) (void)hipStreamSynchronize(copy);
        (void)hipStreamSynchronize(s);
        for (int b = 0; b < 2; ++b) {
            if (stage[b]) (void)hipFree(stage[b]);
            if (ready[b]) (void)hipEventDestroy(ready[b]);
            if (free_[b]) (void)hipEventDestroy(free_[b]);
        }
        if (copy) (void)hipStreamDestroy(copy);
    }
};

}  // namespace

int64_t ingest_chunk_rows(int64_t r0, int64_t nrows) {
    // About 64 MiB of rows per chunk, a whole number of tiles, at least one.
    const int64_t width = r0 + nrows;
    int64_t rows = ((int64_t)64 << 20) / (16 * std::max<int64_t>(width, 1));
    rows = std::max<int64_t>(kT, rows / kT * kT);
    return std::min(rows, nrows);
}

void ingest_rows_host(Z *H, int64_t ldh, const Z *hrows, int64_t ldr, int64_t r0, int64_t nrows,
                      hipStream_t s) {
    if (nrows <= 0) return;
    HostIngest g(s);
    const int64_t width = r0 + nrows;           // widest row of the stripe
    const int64_t chunk = ingest_chunk_rows(r0, nrows);
    CHASE_HIP(hipStreamCreateWithFlags(&g.copy, hipStreamNonBlocking));
    for (int b = 0; b < 2; ++b) {
        CHASE_HIP(hipEventCreateWithFlags(&g.ready[b], hipEventDisableTiming));
        CHASE_HIP(hipEventCreateWithFlags(&g.free_[b], hipEventDisableTiming));
        hipError_t e = hipMalloc(&g.stage[b], (size_t)chunk * width * sizeof(Z));
        if (e != hipSuccess) {
            g.stage[b] = nullptr;
            (void)hipGetLastError();
            throw Error(2, "hipMalloc of the ingestion staging buffer failed");
        }
    }
    int k = 0;
    for (int64_t ra = r0; ra < r0 + nrows; ra += chunk, ++k) {
        const int b = k & 1;
        const int64_t rb = std::min(r0 + nrows, ra + chunk);
        // Chunk k reuses the buffer of chunk k - 2 once its kernel is done.
        if (k >= 2) CHASE_HIP(hipStreamWaitEvent(g.copy, g.free_[b], 0));
        CHASE_HIP(hipMemcpy2DAsync(g.stage[b], (size_t)width * sizeof(Z),
                                   hrows + (ra - r0) * ldr, (size_t)ldr * sizeof(Z),
                                   (size_t)rb * sizeof(Z), (size_t)(rb - ra),
                                   hipMemcpyHostToDevice, g.copy));
        CHASE_HIP(hipEventRecord(g.ready[b], g.copy));
        CHASE_HIP(hipStreamWaitEvent(s, g.ready[b], 0));
        ingest_rows(H, ldh, static_cast<const Z *>(g.stage[b]), width, ra, rb - ra, s);
        CHASE_HIP(hipEventRecord(g.free_[b], s));
    }
    CHASE_HIP(hipStreamSynchronize(s));
}

}  // namespace chase
