/*
 * chase_mi355x.h -- C ABI of an MI355X (gfx950) implementation of ChASE,
 * the Chebyshev Accelerated Subspace iteration Eigensolver used by the
 * modernised Bethe-Salpeter (BSE) solver of Zhang et al., "Solving the
 * Bethe-Salpeter equation on massively parallel architectures"
 * (arXiv:2006.08498).
 *
 * The solver finds the nev algebraically smallest eigenvalues and their
 * eigenvectors of a dense complex Hermitian matrix H of order N (the
 * low-lying excitons; the paper wants full eigenpairs, not eigenvalues
 * only: Sec. "Solving the BSE eigenvalue problem on massively parallel
 * architectures").  nex extra vectors enlarge the search subspace to
 * nev + nex columns (same section; its size changes convergence, supplement
 * Sec. "Dependence of the convergence rate of ChASE on nex").  The phases
 * follow the supplement's list: Lanczos (spectral estimates), Filter
 * (Chebyshev three-term recurrence as repeated HEMM), QR, RR (Rayleigh-Ritz)
 * and Resid (residuals, deflation and locking).
 *
 * Conventions for every call below.
 *  - Pointers named d* are device pointers, h* are host pointers.  The
 *    caller owns all memory passed in; the library never frees it.
 *  - H is complex128, column-major, element (i, j) at dH[i + j*ldh],
 *    ldh >= N, both triangles stored and Hermitian.  H is never written.
 *    (A row-major Hermitian array read as column-major is conj(H) = H^T:
 *    same eigenvalues, conjugated eigenvectors.)
 *  - Eigenvector outputs of the solve calls are column-major N x nev with
 *    leading dimension ldv >= N.  Step-level calls (below the solve calls)
 *    take vector blocks in the solver's internal layout: row-major, element
 *    (i, j) of an N x n block at p[i*ld + j], ld >= n.
 *  - stream is a hipStream_t (NULL = the null stream).  Every call returns
 *    after its work on that stream has completed.
 *  - Status codes are returned; nothing throws across the ABI.  Arguments
 *    are validated before any device work.  On failure chase_last_error()
 *    returns a message (thread-local, valid until the next call on the same
 *    thread).
 *  - Calls on different streams from different threads are re-entrant.
 *  - Results are deterministic: the same inputs, options and seed give the
 *    same bits (no atomics in reductions, fixed reduction order).
 */
#ifndef CHASE_MI355X_H
#define CHASE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* complex128, layout-compatible with std::complex<double> and numpy/torch
 * complex128 */
typedef struct { double re, im; } chase_z;
/* complex64, layout-compatible with numpy/torch complex64 (mixed precision) */
typedef struct { float re, im; } chase_c;

enum chase_status {
    CHASE_PENDING = -1,    /* server: request not finished yet */
    CHASE_OK = 0,
    CHASE_EINVAL = 1,      /* invalid argument */
    CHASE_ENOMEM = 2,      /* device allocation or workspace too small */
    CHASE_EHIP = 3,        /* HIP runtime error */
    CHASE_ENOCONV = 4,     /* max_iter reached; outputs hold the best pairs */
    CHASE_ENONFINITE = 5,  /* NaN/Inf met (e.g. in H) */
    CHASE_EBOUNDS = 6,     /* a Ritz value exceeded the spectral upper bound */
    CHASE_EINTERNAL = 7
};

enum chase_precision {
    CHASE_FP64 = 0,        /* every phase in FP64 */
    CHASE_MIXED = 1        /* filter in FP32 while a vector's residual is
                              above switch_tol, FP64 afterwards */
};

struct chase_info;
typedef int (*chase_iter_fn)(void *user, const struct chase_info *info);

typedef struct chase_opts {
    int32_t precision;        /* chase_precision; default CHASE_FP64 */
    int32_t max_iter;         /* subspace iterations; default 100 */
    int32_t initial_degree;   /* filter degree of the first iteration;
                                 default 20 (capped by degree_max) */
    int32_t degree_extra;     /* steps added to each computed degree;
                                 default 2 */
    int32_t lanczos_steps;    /* Lanczos steps per run; default 25 */
    int32_t lanczos_runs;     /* independent Lanczos runs; default 4 */
    uint64_t seed;            /* start vectors (Philox4x32-10); default 0 */
    double switch_tol;        /* CHASE_MIXED: residual / ||H|| above which a
                                 vector is filtered in FP32 (until FP32 stalls on
                                 it); default 1e-7, about the FP32 floor */
    const chase_z *dV0;       /* optional warm start: v0_cols columns,
                                 column-major, leading dimension N; NULL =
                                 random start.  With a warm start the first
                                 iteration is a Rayleigh-Ritz of the given
                                 block without filtering: its residuals set
                                 the first degrees and its largest Ritz value
                                 the first damped interval, so Lanczos is
                                 needed for the upper bound and ||H|| only
                                 and may be shortened (lanczos_steps 10,
                                 lanczos_runs 1 suffice for a sequence of
                                 nearby matrices) */
    int32_t profile;          /* 1: time every filter launch with HIP events
                                 (fills t_filter_kernels) */
    int32_t graphs;           /* 1 (default): run each Jacobi sweep of the
                                 Rayleigh-Ritz eigensolve as one launch of a
                                 HIP graph (built node by node once per order,
                                 no stream capture); 0: launch the sweep's
                                 kernels one by one.  Same results either
                                 way. */
    /* Optional, called on the host thread running the solve (a server's
     * worker thread for served requests) after every subspace iteration with the record so far (iterations, nconv = locked pairs,
     * counters and phase times; alpha/mu1 of that iteration).  A nonzero
     * return stops the solve after that iteration: the call then returns
     * CHASE_ENOCONV (unless nev pairs are already locked) with the best
     * pairs so far.  NULL = no callback. */
    chase_iter_fn on_iteration;
    void *on_iteration_user;
    /* Sequences of eigenproblems (the solver's original use, Sec. "Solving
     * the BSE eigenvalue problem on massively parallel architectures").
     * v0_cols: columns of dV0 given, 1..nev+nex; 0 (default) = nev+nex; the
     * rest of the start block is random.  out_cols: columns written to dV,
     * nev..nev+nex; 0 (default) = nev.  Columns past nev hold the rest of
     * the final search block (Ritz vectors by ascending Ritz value, same
     * phase normalisation), so that dV of one solve warm-starts the next
     * with v0_cols = out_cols = nev+nex. */
    int32_t v0_cols;
    int32_t out_cols;
    int32_t reserved[2];
} chase_opts;

typedef struct chase_info {
    int32_t iterations;        /* subspace iterations done */
    int32_t nconv;             /* converged (locked) eigenpairs */
    int64_t matvecs_filter;    /* filter column products (H times one
                                  column), the paper's mat-vec count */
    int64_t matvecs_filter_fp32; /* of which in FP32 (CHASE_MIXED) */
    int64_t matvecs_total;     /* filter + Rayleigh-Ritz + Lanczos */
    int64_t filter_launches;   /* filter kernel launches */
    double mu1;                /* lower spectral estimate */
    double mu_ne;              /* Lanczos estimate of lambda_{nev+nex} */
    double alpha;              /* lower end of the damped interval, last
                                  iteration */
    double beta;               /* upper end (spectral upper bound) */
    double hnorm_est;          /* estimate of ||H||_2 used by the tolerance */
    double t_lanczos, t_filter, t_qr, t_rr, t_resid, t_total; /* seconds */
    double t_filter_kernels;   /* sum of filter kernel durations (profile) */
    double filter_flops;       /* algorithmic filter flops, 8 N^2 per
                                  column product (both precisions) */
    double t_shadow;           /* CHASE_MIXED: building the complex64 copy
                                  of H (seconds) */
    double t_filter32_kernels; /* FP32 filter kernel durations (profile) */
    int64_t filter32_launches; /* FP32 filter kernel launches */
    /* profile: every FP64 H-times-block kernel launch of the solve (filter,
     * Lanczos and Rayleigh-Ritz): summed duration, algorithmic flops
     * (8 N^2 per column) and launch count */
    double gemm_time, gemm_flops;
    int64_t gemm_launches;
    /* iterations spent on a whole-block Rayleigh-Ritz (no filter) after the
     * first active pair stalled just above tol behind the locked ones */
    int64_t refinements;
    /* Algorithmic work of each phase over the whole solve (what the method
     * must do, not what the kernels happen to move): flops in real
     * operations (a complex multiply-add is 8) and HBM bytes with every
     * operand read once and every result written once.  Lanczos: k steps of
     * H times r vectors plus the vector updates; filter (both precisions):
     * H (16 or 8 N^2 bytes) once per launch plus the Y, X and W columns;
     * QR: two Gram-Schmidt passes against the locked columns and three
     * CholeskyQR passes; Rayleigh-Ritz: W = H Q, Q^H W and Q Y (the small
     * eigensolve is not counted); residuals: W Y, the norms and the copy
     * back. */
    double lanczos_flops, lanczos_bytes, filter_bytes, qr_flops, qr_bytes, rr_flops,
        rr_bytes, resid_flops, resid_bytes;
} chase_info;

/* Fills *o with the defaults listed above. */
void chase_default_opts(chase_opts *o);

/* Message describing the last failure on this thread ("" if none). */
const char *chase_last_error(void);

/* ------------------------------------------------------------------ solve */

/*
 * Lowest nev eigenpairs of H to residual tolerance tol: every returned pair
 * satisfies ||H v - lambda v||_2 <= tol * ||H||_2 (||H||_2 estimated from
 * below by the Lanczos phase).  h_eigvals: nev doubles, ascending.  dV:
 * N x nev, column-major, leading dimension N, orthonormal columns; in each
 * column the entry of largest modulus (lowest index on ties) is real and
 * positive.  Requires 1 <= nev, 0 <= nex, nev + nex <= N, tol > 0,
 * nev + nex <= 1024 (with nex = 0 and nev < N one extra search vector is
 * carried internally: without it the top wanted vector cannot converge),
 * 1 <= degree_max <= 64 (degrees are even, so an odd degree_max above 1
 * acts as degree_max - 1; degree_max = 1 filters every vector with exactly
 * one step per iteration).  Allocates its own workspace; runs on the null
 * stream.
 */
int chase_solve(const chase_z *dH, int64_t N, int32_t nev, int32_t nex,
                double tol, int32_t degree_max,
                double *h_eigvals, chase_z *dV);

/* Bytes of device workspace chase_solve_ex needs for these sizes. */
size_t chase_workspace_bytes(int64_t N, int32_t nev, int32_t nex,
                             const chase_opts *o);

/*
 * Full form.  h_resid (nev doubles, may be NULL) receives the residual norms
 * ||H v_j - lambda_j v_j||_2.  dV holds nev columns, or o->out_cols when
 * that is set (see chase_opts).  dwork/work_bytes: caller-provided device
 * workspace of at least chase_workspace_bytes() bytes, 256-byte aligned, or
 * NULL/0 to let the library allocate.  o == NULL means defaults.  info may
 * be NULL.  On CHASE_ENOCONV the outputs hold the current best Ritz pairs
 * and info->nconv < nev.
 */
int chase_solve_ex(const chase_z *dH, int64_t N, int64_t ldh,
                   int32_t nev, int32_t nex, double tol, int32_t degree_max,
                   double *h_eigvals, double *h_resid,
                   chase_z *dV, int64_t ldv,
                   void *dwork, size_t work_bytes,
                   void *stream, const chase_opts *o, chase_info *info);

/* ------------------------------------------------------- step-level calls
 * One phase each, on caller-provided blocks (row-major, see above).  They
 * allocate any scratch they need. */

/*
 * One Chebyshev recurrence step over ncols columns (Filter phase, one HEMM
 * with the recurrence folded into its epilogue):
 *     W = a * H Y + b * Y + g * X.
 * dX may be NULL when g == 0.  dW may equal dX (in-place update of the
 * older iterate); dW must not overlap dY.
 */
int chase_filter_step(const chase_z *dH, int64_t N, int64_t ldh,
                      const chase_z *dY, int64_t ldy,
                      const chase_z *dX, int64_t ldx,
                      chase_z *dW, int64_t ldw, int32_t ncols,
                      double a, double b, double g, void *stream);

/* One filter step of a grouped launch: the arguments of chase_filter_step. */
typedef struct chase_filter_call {
    const chase_z *dH;
    int64_t N, ldh;
    const chase_z *dY;
    int64_t ldy;
    const chase_z *dX;
    int64_t ldx;
    chase_z *dW;
    int64_t ldw;
    int32_t ncols;
    double a, b, g;
} chase_filter_call;

/*
 * Several independent filter steps (different H, N and blocks; each with
 * chase_filter_step's contract and checks) in grouped launches: one MFMA
 * grid per distinct tile width holding every step's tiles, then one grid
 * for the split-K reductions.  This is how the server fuses the filter
 * steps of concurrent solves.  Each step's result is bitwise the one
 * chase_filter_step gives.  count in [0, 1024]; the W blocks must not
 * overlap one another or any Y.
 */
int chase_filter_step_group(const chase_filter_call *calls, int32_t count, void *stream);

/*
 * Mixed-precision form (filter with vectors above the switch tolerance):
 * the same step in FP32 on the complex64 copy Hc of H (column-major, ldh)
 * and complex64 row-major blocks, FP32 MFMA with FP32 accumulation.  dX may
 * be NULL when g == 0; dW may equal dX, must not overlap dY.
 */
int chase_filter_step_c(const chase_c *dHc, int64_t N, int64_t ldh,
                        const chase_c *dY, int64_t ldy, const chase_c *dX,
                        int64_t ldx, chase_c *dW, int64_t ldw, int32_t ncols,
                        float a, float b, float g, void *stream);

/* Complex64 copy of H (each part rounded to nearest FP32), column-major
 * with leading dimension ldc >= N; the solver builds it once per
 * CHASE_MIXED solve. */
int chase_shadow_c(const chase_z *dH, int64_t N, int64_t ldh, chase_c *dHc,
                   int64_t ldc, void *stream);

/*
 * The whole Chebyshev filter with per-vector degrees on an N x n block,
 * in place: column j becomes C_m(L) v_j / C_m(t0), m = h_degrees[j],
 * L = (H - cI)/e, t0 = (mu1 - c)/e, c = (alpha+beta)/2, e = (beta-alpha)/2.
 * h_degrees: n integers, ascending, each 1 or even in [2, 64].  Returns the
 * number of column products in *matvecs (may be NULL).
 */
int chase_filter(const chase_z *dH, int64_t N, int64_t ldh,
                 chase_z *dV, int64_t ldv, int32_t n,
                 const int32_t *h_degrees, double mu1, double alpha,
                 double beta, int64_t *matvecs, void *stream);

/* One filter call (as chase_filter) of a batch run by chase_filter_fused. */
typedef struct chase_filter_job {
    const chase_z *dH;
    int64_t N, ldh;
    chase_z *dV;                /* N x n row-major block, filtered in place */
    int64_t ldv;
    int32_t n;
    const int32_t *h_degrees;   /* n degrees, ascending, each 1 or even in [2, 64] */
    double mu1, alpha, beta;
} chase_filter_job;

/*
 * The whole filter calls of several eigenproblems (each with chase_filter's
 * contract and checks; different H, N and blocks) run by one persistent
 * kernel: the recurrence steps of all jobs are dealt out as tiles to the
 * GPU's workgroups as soon as each job's previous step is complete, so the
 * steps of small problems share the GPU without a launch per step.  This is
 * the fused form the server uses for concurrent solves
 * (CHASE_SERVER_FUSE_FILTER).  Each job's result is bitwise the one
 * chase_filter gives it alone.  count in [0, 4096]; the blocks must not
 * overlap one another.  *matvecs (may be NULL) receives the total column
 * products.  Allocates a copy of each block and its scratch.
 */
int chase_filter_fused(const chase_filter_job *jobs, int32_t count, int64_t *matvecs,
                       void *stream);

/*
 * k Lanczos steps from each of the r columns of dV0 (N x r, need not be
 * normalised; not modified).  h_alpha, h_beta: k*r doubles each, row-major
 * [step][run]; T of run q is tridiag(alpha[:, q]; beta[0:k-1, q]) and
 * beta[k-1, q] is the norm of the last residual.
 */
int chase_lanczos(const chase_z *dH, int64_t N, int64_t ldh,
                  const chase_z *dV0, int64_t ldv0, int32_t r, int32_t k,
                  double *h_alpha, double *h_beta, void *stream);

/*
 * Spectral estimates from Lanczos output (host only): out[0] = mu1
 * (smallest Ritz value), out[1] = mu_ne (spectral-density estimate of
 * lambda_ne), out[2] = upper bound (largest Ritz value + last beta, max over
 * runs), out[3] = largest |Ritz value| (estimate of ||H||_2 from below).
 */
int chase_lanczos_bounds(const double *h_alpha, const double *h_beta,
                         int32_t k, int32_t r, int64_t N, int32_t ne,
                         double *out4);

/*
 * QR phase: orthonormalise columns [nlocked, n) of the N x n block dV in
 * place, against the (orthonormal, unchanged) columns [0, nlocked) and
 * among themselves, so that span is kept: two classical Gram-Schmidt passes
 * against the locked columns, then shifted CholeskyQR3 with column
 * scaling.  The result equals Q of V_active = Q R with diag(R) > 0.
 * Requires 1 <= n <= min(N, 1024), 0 <= nlocked <= n, ldv >= n.  A
 * numerically rank-deficient active block (a Cholesky breakdown) returns
 * CHASE_EINTERNAL with the dependent column named in chase_last_error();
 * the block is then partly transformed.  (Inside a solve the column is
 * replaced by a fresh random vector and the QR redone instead.)
 */
int chase_qr(chase_z *dV, int64_t N, int64_t ldv, int32_t n,
             int32_t nlocked, void *stream);

/*
 * RR phase on the orthonormal N x n block dQ: G = Q^H H Q, G = Y Theta Y^H
 * (Theta ascending), Q <- Q Y in place.  h_theta: n doubles.  If h_resid is
 * not NULL it receives ||H q_j - theta_j q_j||_2 (Resid phase).
 */
int chase_rayleigh_ritz(const chase_z *dH, int64_t N, int64_t ldh,
                        chase_z *dQ, int64_t ldq, int32_t n,
                        double *h_theta, double *h_resid, void *stream);

/*
 * Resid phase: h_resid[j] = ||H v_j - h_theta[j] v_j||_2 for the N x n
 * block dV.
 */
int chase_residuals(const chase_z *dH, int64_t N, int64_t ldh,
                    const chase_z *dV, int64_t ldv, int32_t n,
                    const double *h_theta, double *h_resid, void *stream);

/*
 * Dense Hermitian eigensolver for the reduced problem (on the device,
 * cyclic Jacobi): dG n x n row-major (leading dimension n), not modified;
 * h_w: n eigenvalues ascending; dY: n x n row-major eigenvectors (columns).
 * 1 <= n <= 1024.  Sweeps run until the off-diagonal norm is below
 * 1e-15 of the whole or stops falling below 1e-12 of it (the rounding
 * floor); if neither happens within 30 sweeps (environment variable
 * CHASE_JACOBI_MAX_SWEEPS overrides the cap, for diagnostics) the call
 * returns CHASE_EINTERNAL, and so does a solve whose Rayleigh-Ritz phase
 * meets that.  Scratch (4 n^2 complex) is allocated per call.
 */
int chase_heevj(const chase_z *dG, int32_t n, double *h_w, chase_z *dY,
                void *stream);

/*
 * chase_heevj without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels in the same order, so
 * the same bits as chase_heevj, with the working copy of G, the Jacobi
 * buffers and the eigenvalues (4 n^2 complex + n doubles) in a static
 * device array of the library of 16 MiB + 64 KiB, which each GPU the
 * library runs on holds until the process ends.  1 <= n <= 512; a larger n
 * returns CHASE_EINVAL (use chase_heevj).  Calls no hipMalloc, hipFree or
 * other allocating routine.  The array keeps the last call's contents
 * (nothing in it needs clearing: every entry a call reads it writes first).
 * Overlapping calls on one GPU would race on the array, so the library
 * serialises them (the call is synchronous); separate processes hold
 * separate arrays.  Same arguments and results as chase_heevj.
 */
int chase_heevj_noalloc(const chase_z *dG, int32_t n, double *h_w, chase_z *dY,
                        void *stream);

/*
 * Filter degrees (host only): for each of n vectors with Ritz value
 * h_theta[j] and residual h_resid[j], the smallest m with
 * rho_j^m >= resid_j / tol_abs (rho_j of the supplement's Eq. S1 on the
 * interval [alpha, beta]) plus extra, clamped to [2, degree_max] and made
 * even; 2 for converged vectors; 1 for every vector when degree_max is 1.
 */
int chase_degrees(const double *h_theta, const double *h_resid, int32_t n,
                  double tol_abs, double alpha, double beta,
                  int32_t degree_max, int32_t extra, int32_t *h_degrees);

/*
 * nex for a matrix of a series by linear interpolation in the energy cutoff
 * (supplement Eq. S2, Sec. "Optimization of the nex value"): nex_low at
 * e_low, nex_high at e_high, rounded to the nearest integer (halves away
 * from zero); e outside [e_low, e_high] extrapolates, and the result is at
 * least 0.  Host only.  Returns -1 (with chase_last_error set) unless
 * e_high > e_low, both finite, e finite and nex_low, nex_high >= 0.  The
 * supplement's Table S10 is reproduced with e_high = 14.32 eV, not the
 * printed 12.82 (the largest cutoff of the table).
 */
int32_t chase_nex_linear(int32_t nex_low, int32_t nex_high, double e_low, double e_high,
                         double e);

/* ------------------------------------------------------------ ingesting H
 * The paper reads H as stripes of rows of its lower half and then fills the
 * upper half from the ranks holding the transposed parts (Sec. "Matrix
 * generation and the I/O challenge").  These calls build the column-major
 * Hermitian H that the solve calls read from such stripes, or complete H in
 * place from one stored triangle.  The result is Hermitian to the last bit
 * with a real diagonal (the imaginary part of a stored diagonal entry is
 * dropped).  All require 1 <= N <= 180000 and ldh >= N.
 */

/*
 * Rows [r0, r0 + nrows) of the lower triangle, row-major in device memory:
 * row r at dRows + (r - r0)*ldr, of which columns 0..r are read (entries
 * right of the diagonal are never read).  Writes H(r, c) and
 * H(c, r) = conj(H(r, c)) for c < r, and H(r, r) = its real part.  Stripes
 * may come in any order; once they cover rows 0..N-1, dH is complete.
 * Requires r0 >= 0, nrows >= 0, r0 + nrows <= N, ldr >= r0 + nrows, dH and
 * dRows not NULL when nrows > 0; dRows must not overlap dH.
 */
int chase_ingest_rows(chase_z *dH, int64_t N, int64_t ldh, const chase_z *dRows,
                      int64_t ldr, int64_t r0, int64_t nrows, void *stream);

/*
 * The same from host memory hRows (same layout), streamed in chunks of rows
 * through two device staging buffers that the call allocates (about 64 MiB
 * each) and frees: the host-to-device copy of one chunk, on a stream of the
 * call's own, overlaps the ingestion of the previous chunk on `stream`.
 * Page-locked hRows (hipHostMalloc, torch pin_memory) moves at the PCIe
 * rate; pageable memory works, more slowly.  CHASE_ENOMEM if the staging
 * buffers cannot be allocated.
 */
int chase_ingest_rows_host(chase_z *dH, int64_t N, int64_t ldh, const chase_z *hRows,
                           int64_t ldr, int64_t r0, int64_t nrows, void *stream);

/*
 * H in place from its lower (uplo = 'L') or upper (uplo = 'U') triangle,
 * diagonal included: the other strict triangle becomes the conjugate
 * transpose and the diagonal's imaginary part 0.
 */
int chase_hermitian_complete(chase_z *dH, int64_t N, int64_t ldh, int32_t uplo,
                             void *stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent eigenproblems on one GPU (no source
 * in the paper, which solves one matrix at a time; its workflows solve
 * series of matrices, Sec. "A practical case: converging exciton-binding
 * energy in naphthalene").  Requests of uneven N are admitted first-fit in
 * arrival order as soon as a slot is free and their device footprint (H
 * unless the caller holds it, the solver workspace and the eigenvector
 * output) fits the memory budget; admitted requests run concurrently, one
 * HIP stream per slot, with H and the subspace resident until the result is
 * collected.  A request's result is bitwise the same alone and in the mix.
 */
typedef struct chase_server chase_server;

/* Produces H for a request at admission: writes the N x N column-major
 * complex128 matrix (leading dimension ldh) into dH (device memory the
 * server owns) with work enqueued on `stream`; returns 0 on success.  Called
 * from a server thread. */
typedef int (*chase_fill_fn)(chase_z *dH, int64_t N, int64_t ldh, void *user,
                             void *stream);

/* Server flags. */
enum {
    /* Fuse the FP64 filter steps of concurrent small solves (N <= 8192,
     * whose own launches underfill the GPU): each hands its filter call to
     * one persistent kernel of the server (the engine behind
     * chase_filter_fused), which deals out the tiles of all handed-over
     * calls as each call's previous step completes, instead of one launch
     * per step per solve; larger solves launch their own.  Results are
     * bitwise the same either way. */
    CHASE_SERVER_FUSE_FILTER = 1,
    /* Admission order: among the queued requests that fit, the one with
     * the least estimated work (N^2 (nev + nex)) first, instead of arrival
     * order; a request that has waited longer than the aging time (30 s by
     * default, chase_server_set_aging) is admitted first, in arrival order,
     * so large requests are not starved.  Lowers the median latency of an
     * overloaded server at the cost of its largest requests. */
    CHASE_SERVER_SHORTEST_FIRST = 2
};

/* hbm_budget_bytes: device memory the server may allocate (0 = free memory
 * minus a reserve); max_slots: concurrent solves (1..64); flags: a
 * combination of CHASE_SERVER_FUSE_FILTER and CHASE_SERVER_SHORTEST_FIRST
 * (0 = arrival order, no fusion).  NULL on failure
 * (chase_server_last_error()). */
chase_server *chase_server_create(size_t hbm_budget_bytes, int32_t max_slots,
                                  uint32_t flags);

/* Queues a request.  H is a host matrix (copied now, uploaded at admission,
 * counted in the footprint) when is_device == 0, else a caller-owned device
 * matrix with ldh == N that must stay valid and unmodified until the
 * request is polled (not counted).  The server reads a device H on a
 * stream of its own that is not ordered after the caller's streams: the
 * work that writes H must have completed before this call (synchronise the
 * stream that produced it).  Arguments and options are checked as by
 * chase_solve_ex (no warm start; out_cols 0 or nev) before the request is
 * queued: CHASE_EINVAL on a bad one.  Returns CHASE_ENOMEM if the footprint
 * alone exceeds the budget. */
int chase_server_submit(chase_server *srv, const chase_z *H, int is_device,
                        int64_t N, int64_t ldh, int32_t nev, int32_t nex,
                        double tol, int32_t degree_max, const chase_opts *o,
                        uint64_t *ticket);

/* Queues a request whose H is produced at admission by `fill` (counted in
 * the footprint). */
int chase_server_submit_fill(chase_server *srv, chase_fill_fn fill, void *user,
                             int64_t N, int32_t nev, int32_t nex, double tol,
                             int32_t degree_max, const chase_opts *o,
                             uint64_t *ticket);

/* CHASE_PENDING while the request is queued or running.  Otherwise copies
 * the results (eigenvalues ascending into h_eigvals, residuals into h_resid
 * if not NULL, eigenvectors column-major into dV with ldv >= N, info if not
 * NULL, and if h_times3 is not NULL: seconds queued, seconds on the GPU,
 * latency from submission to completion), releases the request and returns
 * its status (CHASE_OK, CHASE_ENOCONV or the error).  The eigenvectors are
 * copied on a stream of the server's own, complete when the call returns;
 * that copy is not ordered after the caller's streams, so no queued work
 * may still use dV.  One poll collects a result: a concurrent poll of the
 * same ticket gets CHASE_EINVAL (so does a NULL dV or ldv < N, after which
 * the result can still be collected). */
int chase_server_poll(chase_server *srv, uint64_t ticket, double *h_eigvals,
                      double *h_resid, chase_z *dV, int64_t ldv,
                      chase_info *info, double *h_times3);

/* Blocks until the request is done (timeout_s < 0: no timeout); CHASE_OK
 * when done, CHASE_PENDING on timeout. */
int chase_server_wait(chase_server *srv, uint64_t ticket, double timeout_s);

/* Memory in use and its peak (bytes), running and peak running requests,
 * queued requests.  Any pointer may be NULL. */
int chase_server_stats(chase_server *srv, size_t *bytes_in_use,
                       size_t *peak_bytes, int32_t *running,
                       int32_t *peak_running, int32_t *queued);

/* With CHASE_SERVER_SHORTEST_FIRST: the wait (seconds, >= 0) after which a
 * queued request is admitted in arrival order. */
int chase_server_set_aging(chase_server *srv, double seconds);

/* With CHASE_SERVER_FUSE_FILTER: launches of the persistent filter kernel
 * so far (it runs while filter calls are in flight and stops when none is
 * left) and the filter steps it ran; both 0 without fusion. */
int chase_server_fusion_stats(chase_server *srv, int64_t *ticks, int64_t *steps);

/* Message for the last server call that failed on this thread. */
const char *chase_server_last_error(void);

/* Drops queued requests, waits for running ones, frees everything. */
void chase_server_destroy(chase_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* CHASE_MI355X_H */
