// The ChASE driver on one stream.
#pragma once

#include "../../include/chase_mi355x.h"
#include "common.h"

#include <vector>

namespace chase {

// Device workspace carved from one allocation (offsets in bytes).
struct Layout {
    int64_t N;
    int ne, r, k;
    size_t V, B1, W, T, fpart, gpart, G, Bq, cwork, Y, jwork, theta, resid,
        npart, perm, info, Lv, Lvp, Lw, Lal, Lbe, Lpart;
    // CHASE_MIXED only (size 0 otherwise): complex64 shadow of H, two FP32
    // vector blocks and the FP32 split-K partials.
    size_t Hc, Vc, Bc, fpart32;
    bool mixed;
    size_t total;
};
int internal_nex(int64_t N, int nev, int nex);
Layout make_layout(int64_t N, int nev, int nex, const chase_opts &o);

// Where a solve sends the FP64 filter steps of one iteration instead of
// launching them itself (the server's cross-request fusion).  run() must
// leave the steps ordered after the work already on `s`, and the work
// enqueued on `s` afterwards ordered after them.
struct FilterSink {
    virtual void run(std::vector<FilterCall> &&steps, hipStream_t s) = 0;
    virtual ~FilterSink() = default;
};

struct Problem {
    const Z *H;
    int64_t N, ldh;
    int nev, nex;
    double tol;
    int degree_max;
    chase_opts opts;
    FilterSink *sink = nullptr;
};

struct Result {
    std::vector<double> eigvals, resid;
    chase_info info;
    int status;   // CHASE_OK or CHASE_ENOCONV
};

// Runs the solve; eigenvectors (column-major, ldv) go to dV.
Result solve(const Problem &p, void *dwork, Z *dV, int64_t ldv,
             hipStream_t s);

// The filter's GEMMs for one iteration, in order (see filter_block).
std::vector<FilterCall> filter_steps(const Z *H, int64_t ldh, int64_t N, Z *V, Z *B1,
                                     int64_t ld, int n, const int *deg, double mu1,
                                     double alpha, double beta, Z *fpart);

// Argument checks of a solve, before any device work (throw Error with
// CHASE_EINVAL): sizes, tol, degree_max and the options.  Shared by the
// solve calls and the server's submissions.
void validate_sizes(int64_t N, int32_t nev, int32_t nex);
void validate_opts(const chase_opts &o);
void validate_problem(int64_t N, int32_t nev, int32_t nex, double tol, int32_t degree_max,
                      const chase_opts &o);

// Copies the leading degree-1 columns of a filtered block (deg ascending)
// from B1, where a one-step recurrence leaves them, back to V.
void finish_degree_one(Z *V, const Z *B1, int64_t ld, int64_t N, int n, const int *deg,
                       hipStream_t s);

// Step-level helpers shared with the C ABI.
void filter_block(const Z *H, int64_t ldh, int64_t N, Z *V, Z *B1, int64_t ld,
                  int n, const int *deg, double mu1, double alpha, double beta,
                  Z *fpart, hipStream_t s, std::vector<hipEvent_t> *prof);
void filter32_block(const C *Hc, int64_t N, C *V, C *B1, int64_t ld, int n,
                    const int *deg, double mu1, double alpha, double beta,
                    C *fpart, hipStream_t s, std::vector<hipEvent_t> *prof);
void qr_block(Z *V, Z *B1, int64_t ld, int64_t N, int L, int ne, Z *G, Z *Bq,
              Z *cwork, Z *gpart, int *dinfo, hipStream_t s);
void rr_block(const Z *H, int64_t ldh, int64_t N, Z *Q, Z *W, Z *T, Z *B1,
              int64_t ld, int n, Z *G, Z *Y, Z *jwork, double *theta,
              double *resid, Z *fpart, Z *gpart, double *npart, double *hwork,
              hipStream_t s);

}  // namespace chase
