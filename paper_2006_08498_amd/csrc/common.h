// Internal declarations shared by the HIP sources of libchase_mi355x.
#pragma once

#include <hip/hip_runtime.h>

#include "k_filter_plan.h"

#include <cstdint>
#include <stdexcept>
#include <string>
#include <algorithm>
#include <utility>
#include <vector>

namespace chase {

using Z = double2;   // complex128: .x = real, .y = imaginary
using C = float2;    // complex64 (mixed-precision filter)

// Error carried up to the C ABI, which turns it into a status code.
struct Error : std::runtime_error {
    int status;
    Error(int st, const std::string &m) : std::runtime_error(m), status(st) {}
};

#define CHASE_HIP(call)                                                       \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            throw ::chase::Error(3, std::string(#call) + ": " +              \
                                        hipGetErrorString(e_));               \
    } while (0)

inline void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw Error(3, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- kernels
// All vector blocks are row-major (element (i, j) at p[i*ld + j]); H is
// column-major.  Every launcher enqueues on `s` and returns immediately.

// Filter GEMM: W[:, 0:n] = a*H*Y + b*Y + g*X (X may be null when g == 0;
// W may alias X).  `part` is scratch for split-K partial sums of
// filter_partial_elems(N, n) elements (may be null if that is 0).

void filter_gemm(const Z *H, int64_t ldh, int64_t N, const Z *Y, int64_t ldy,
                 const Z *X, int64_t ldx, Z *W, int64_t ldw, int n, double a,
                 double b, double g, Z *part, hipStream_t s,
                 hipEvent_t after_mfma = nullptr);

// One filter GEMM of a grouped launch (the same contract as filter_gemm).
struct FilterCall {
    const Z *H;
    int64_t ldh, N;
    const Z *Y;
    int64_t ldy;
    const Z *X;
    int64_t ldx;
    Z *W;
    int64_t ldw;
    int n;
    double a, b, g;
    Z *part;
};
// Several independent filter GEMMs (different H, sizes and buffers) in as
// few launches as possible: one MFMA launch per distinct tile width and one
// reduction launch for the split ones (per round of column chunks).  Each
// call keeps the column chunks and tile plans filter_gemm gives it alone,
// so its result is bitwise the same as a filter_gemm call.
void filter_gemm_group(const FilterCall *calls, int count, hipStream_t s);

// Ingesting H (k_ingest.hip).  ingest_rows: rows [r0, r0 + nrows) of the
// lower triangle, row-major in device memory (row r at rows + (r - r0)*ldr,
// columns 0..r read), written into both triangles of the column-major H with
// a real diagonal.  ingest_rows_host: the same from host memory, streamed
// through two device staging buffers of ingest_chunk_rows() rows so that the
// copy of one chunk overlaps the kernel of the previous; returns after the
// work on s is done.  hermitian_complete: H in place from its lower (or
// upper) triangle.
void ingest_rows(Z *H, int64_t ldh, const Z *rows, int64_t ldr, int64_t r0, int64_t nrows,
                 hipStream_t s);
int64_t ingest_chunk_rows(int64_t r0, int64_t nrows);
void ingest_rows_host(Z *H, int64_t ldh, const Z *hrows, int64_t ldr, int64_t r0, int64_t nrows,
                      hipStream_t s);
void hermitian_complete(Z *H, int64_t ldh, int64_t N, bool lower, hipStream_t s);

// FP32 filter GEMM on the complex64 shadow Hc (mixed precision), same
// contract as filter_gemm; partials: filter32_partial_elems(N, n) complex64.
void filter32_gemm(const C *H, int64_t ldh, int64_t N, const C *Y, int64_t ldy,
                   const C *X, int64_t ldx, C *W, int64_t ldw, int n, float a,
                   float b, float g, C *part, hipStream_t s,
                   hipEvent_t after_mfma = nullptr);
// Conversions: H (column-major) -> complex64 shadow; row-major blocks.
void z2c_matrix(const Z *H, int64_t ldh, C *Hc, int64_t ldc, int64_t N, hipStream_t s);
void z2c_block(const Z *V, int64_t ldv, C *Vc, int64_t ldc, int64_t N, int n,
               hipStream_t s);
void c2z_block(const C *Vc, int64_t ldc, Z *V, int64_t ldv, int64_t N, int n,
               hipStream_t s);

// C (p x q, row-major ldc) = A^H B over N rows; A: N x p, B: N x q.
// `part` holds gram_partial_elems(N, p, q) elements of split-K partials.
// herm (requires A = B): only the tiles on and above the diagonal are
// computed and C is made Hermitian to the last bit (real diagonal).
size_t gram_partial_elems(int64_t N, int p, int q);
void gram(const Z *A, int64_t lda, const Z *B, int64_t ldb, int64_t N, int p,
          int q, Z *C, int64_t ldc, Z *part, hipStream_t s, bool herm = false);

// C (N x q) = alpha * A (N x p) * B (p x q, row-major ldb) + beta * C0.
// C0 may alias C or be null (beta == 0).  C must not overlap A.  upper: B is
// upper triangular (rows below each column's diagonal are skipped).
void tsmm(const Z *A, int64_t lda, const Z *B, int64_t ldb, int64_t N, int p,
          int q, double alpha, const Z *C0, int64_t ldc0, double beta, Z *C,
          int64_t ldc, hipStream_t s, bool upper = false);

// Column norms of (V - V2 * diag(theta)) or of V (V2 == null); deterministic
// two-pass reduction.  out: n doubles on the device.  part: norm_partial_elems.
size_t norm_partial_elems(int64_t N, int n);
void col_norms(const Z *V, int64_t ldv, const Z *V2, int64_t ldv2,
               const double *theta, int64_t N, int n, double *part,
               double *out, hipStream_t s);

// Row-major block copies and layout changes.
void copy_block(const Z *src, int64_t lds, Z *dst, int64_t ldd, int64_t N,
                int n, hipStream_t s);
// dst[i*ldd + j] = src[i*lds + perm[j]]  (perm on the device)
void permute_cols(const Z *src, int64_t lds, Z *dst, int64_t ldd, int64_t N,
                  int n, const int *perm, hipStream_t s);
// Column-major (ldc) <-> row-major (ldr), N x n.
void colmajor_to_rowmajor(const Z *src, int64_t ldc, Z *dst, int64_t ldr,
                          int64_t N, int n, hipStream_t s);
void rowmajor_to_colmajor(const Z *src, int64_t ldr, Z *dst, int64_t ldc,
                          int64_t N, int n, hipStream_t s);
// Phase normalisation (largest-modulus entry real positive) of each column
// of a row-major block, written column-major to dst.  scratch: 2*n*nblk.
size_t phase_scratch_elems(int64_t N, int n);
void phase_normalise_out(const Z *V, int64_t ldv, int64_t N, int n, Z *dst,
                         int64_t ldd, double *scratch, hipStream_t s);

// Complex Gaussian block (E|z|^2 = 1) from Philox4x32-10 keyed by seed,
// counter (i, j, stream, 0); row-major ld.
void random_block(Z *V, int64_t ld, int64_t N, int n, uint64_t seed,
                  uint32_t stream, hipStream_t s);

// Non-finite check of the column-major H: *flag (device int) set to 1 if any
// entry is NaN/Inf.  The caller zeroes the flag.
void check_finite(const Z *H, int64_t ldh, int64_t N, int *flag, hipStream_t s);

// Lanczos: one fused update per run after w = H v (r runs are columns of
// row-major N x r blocks):  alpha = Re v^H w;  w -= alpha v + beta_prev vp;
// beta = ||w||;  vp <- v;  v <- w / beta.  Writes alpha/beta for `step`.
// If `normalise_only`, just sets v <- v0 / ||v0|| and vp <- 0.
size_t lanczos_scratch_elems(int64_t N, int r);
void lanczos_update(Z *v, Z *vp, Z *w, int64_t ld, int64_t N, int r,
                    double *alpha, double *beta, int step, int normalise_only,
                    double *scratch, hipStream_t s);

// ------------------------------------------------- small dense (n <= 1024)
// G (n x n Hermitian, row-major ld n, not modified) -> B = D * L^{-H}
// (row-major n x n, the right factor for V <- V B), L the lower Cholesky
// factor of D G D + shift I with D = diag(1/sqrt(G_jj)).  work:
// chol_work_elems(n) complex elements.  info: device int, set to
// 1 + column on a non-positive pivot, else 0.
size_t chol_work_elems(int n);
void chol_qr_factor(const Z *G, int n, double shift, Z *B, Z *work, int *info,
                    hipStream_t s);
// Reduced Hermitian eigenproblem by cyclic Jacobi.  A: n x n row-major
// (overwritten).  On return w (device, ascending) and Y (row-major, columns
// are eigenvectors).  work: jacobi_work_elems(n) complex elements.
// Jacobi sweeps as HIP graphs (one per order n and buffer set, one for
// each ping-pong parity, built node by node) replayed once per sweep;
// owned by one solve, which passes it to every jacobi_eig call.
struct JacobiGraphs {
    struct Entry {
        int n;
        const void *A, *work;
        hipGraphExec_t exec[2];
        int last_sweeps;   // sweeps the previous eigensolve of this order took
    };
    hipStream_t used = nullptr;  // stream the graphs were launched on
    std::vector<Entry> entries;
    JacobiGraphs() = default;
    JacobiGraphs(const JacobiGraphs &) = delete;
    JacobiGraphs &operator=(const JacobiGraphs &) = delete;
    ~JacobiGraphs();
};
size_t jacobi_work_elems(int n);
// hstatus (pinned host int, optional): for the one-launch path (n <=
// kJacobiLds) the convergence status is copied there and not checked, so
// the call returns without waiting for the stream; the caller passes it to
// jacobi_check_status after its next synchronisation.
void jacobi_eig(Z *A, int n, double *w, Z *Y, Z *work, double *hwork,
                hipStream_t s, JacobiGraphs *graphs = nullptr, int *hstatus = nullptr);
void jacobi_check_status(int n, int status);
// The same eigensolve (no sweep graphs) with every buffer in a static
// device array of the library, so that it allocates nothing: G (n x n,
// not modified) -> h_w (host, ascending) and Y; 1 <= n <= kNoAllocMaxOrder.
// Synchronous; concurrent calls on one GPU are serialised.
constexpr int kNoAllocMaxOrder = 512;
void jacobi_eig_noalloc(const Z *G, int n, double *h_w, Z *Y, hipStream_t s);
// Symmetrise: G <- (G + G^H)/2, real diagonal.
void hermitise(Z *G, int n, hipStream_t s);

}  // namespace chase
