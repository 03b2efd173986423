// The ChASE driver on one HIP stream (Lanczos -> loop {Filter, QR, RR,
// Resid, lock}), following the phase list of the paper's supplement.  All
// vector work stays on the device; per iteration only 2*(nev+nex) doubles
// (Ritz values and residual norms) come back to the host, which then picks
// the locks, the filter interval and the per-vector degrees.
#include "solver.h"

#include "control.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>

namespace chase {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// With nex = 0 the largest Ritz value is the top wanted one, so the damped
// interval [alpha, beta] would start at or above lambda_nev and the last
// wanted vector would never separate from lambda_{nev+1}: one extra vector
// is then carried internally (unless nev = N, where the subspace is the
// whole space and Rayleigh-Ritz is exact).
int internal_nex(int64_t N, int nev, int nex) {
    return (nex == 0 && nev < N) ? 1 : nex;
}

Layout make_layout(int64_t N, int nev, int nex, const chase_opts &o) {
    Layout L{};
    L.N = N;
    L.ne = nev + internal_nex(N, nev, nex);
    L.r = std::max(1, o.lanczos_runs);
    L.k = (int)std::max<int64_t>(1, std::min<int64_t>(o.lanczos_steps, N));
    const int ne = L.ne;
    const size_t zb = sizeof(Z);
    size_t fpart = filter_partial_elems(N, L.r);
    for (int n = 1; n <= ne; ++n) fpart = std::max(fpart, filter_partial_elems(N, n));
    size_t gpart = 0;
    for (int n = 1; n <= ne; ++n) {
        gpart = std::max(gpart, gram_partial_elems(N, n, n));
        if (n < ne) gpart = std::max(gpart, gram_partial_elems(N, ne - n, n));
    }
    const size_t nn = (size_t)ne * ne;
    const size_t npart = std::max(norm_partial_elems(N, ne), phase_scratch_elems(N, ne));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align256(off + std::max<size_t>(bytes, 1));
        return at;
    };
    L.V = take((size_t)N * ne * zb);
    L.B1 = take((size_t)N * ne * zb);
    L.W = take((size_t)N * ne * zb);
    L.T = take((size_t)N * ne * zb);
    L.fpart = take(fpart * zb);
    L.gpart = take(gpart * zb);
    L.G = take(nn * zb);
    L.Bq = take(nn * zb);
    L.cwork = take(chol_work_elems(ne) * zb);
    L.Y = take(nn * zb);
    L.jwork = take(jacobi_work_elems(ne) * zb);
    L.theta = take((size_t)ne * sizeof(double));
    L.resid = take((size_t)ne * sizeof(double));
    L.npart = take(npart * sizeof(double));
    L.perm = take((size_t)ne * sizeof(int));
    L.info = take(4 * sizeof(int));
    L.Lv = take((size_t)N * L.r * zb);
    L.Lvp = take((size_t)N * L.r * zb);
    L.Lw = take((size_t)N * L.r * zb);
    L.Lal = take((size_t)L.k * L.r * sizeof(double));
    L.Lbe = take((size_t)L.k * L.r * sizeof(double));
    L.Lpart = take(lanczos_scratch_elems(N, L.r) * sizeof(double));
    L.mixed = o.precision == CHASE_MIXED;
    L.Hc = L.Vc = L.Bc = L.fpart32 = 0;
    if (L.mixed) {
        size_t f32 = 0;
        for (int n = 1; n <= ne; ++n) f32 = std::max(f32, filter32_partial_elems(N, n));
        L.Hc = take((size_t)N * N * sizeof(C));
        L.Vc = take((size_t)N * ne * sizeof(C));
        L.Bc = take((size_t)N * ne * sizeof(C));
        L.fpart32 = take(f32 * sizeof(C));
    }
    L.total = off;
    return L;
}

// ------------------------------------------------------------ Filter
// Columns sorted by ascending degree (1 or even); column j stops after
// deg[j] steps, so step s runs on the suffix of columns with deg >= s.  Two
// buffers: V holds Y_0 and every even iterate, B1 every odd iterate, each
// step writing over the older iterate in place.  Even-degree columns end in
// V; the leading degree-1 columns end in B1 and are copied back
// (finish_degree_one).
std::vector<FilterCall> filter_steps(const Z *H, int64_t ldh, int64_t N, Z *V, Z *B1,
                                     int64_t ld, int n, const int *deg, double mu1,
                                     double alpha, double beta, Z *fpart) {
    std::vector<FilterCall> out;
    if (n <= 0) return out;
    const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
    const double sigma1 = e / (mu1 - c);
    const double tau = 2.0 / sigma1;
    const int mmax = deg[n - 1];
    auto step = [&](const Z *Y, const Z *X, Z *W, int cols, double a, double b, double g) {
        out.push_back(FilterCall{H, ldh, N, Y, ld, X, ld, W, ld, cols, a, b, g, fpart});
    };
    {
        const double a = sigma1 / e;
        step(V, nullptr, B1, n, a, -c * a, 0.0);
    }
    double sprev = sigma1;
    int first = 0;
    for (int st = 2; st <= mmax; ++st) {
        const double sigma = 1.0 / (tau - sprev);
        const double a = 2.0 * sigma / e;
        const double g = -sprev * sigma;
        while (first < n && deg[first] < st) ++first;
        const int cols = n - first;
        if (st % 2 == 0) step(B1 + first, V + first, V + first, cols, a, -c * a, g);
        else step(V + first, B1 + first, B1 + first, cols, a, -c * a, g);
        sprev = sigma;
    }
    return out;
}

static int degree_one_count(const int *deg, int n) {
    int n1 = 0;
    while (n1 < n && deg[n1] == 1) ++n1;
    return n1;
}

void finish_degree_one(Z *V, const Z *B1, int64_t ld, int64_t N, int n, const int *deg,
                       hipStream_t s) {
    copy_block(B1, ld, V, ld, N, degree_one_count(deg, n), s);
}

void filter_block(const Z *H, int64_t ldh, int64_t N, Z *V, Z *B1, int64_t ld,
                  int n, const int *deg, double mu1, double alpha, double beta,
                  Z *fpart, hipStream_t s, std::vector<hipEvent_t> *prof) {
    for (const FilterCall &f :
         filter_steps(H, ldh, N, V, B1, ld, n, deg, mu1, alpha, beta, fpart)) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (prof) {
            CHASE_HIP(hipEventCreate(&e0));
            CHASE_HIP(hipEventCreate(&e1));
            CHASE_HIP(hipEventCreate(&e2));
            CHASE_HIP(hipEventRecord(e0, s));
        }
        filter_gemm(f.H, f.ldh, f.N, f.Y, f.ldy, f.X, f.ldx, f.W, f.ldw, f.n, f.a, f.b, f.g,
                    f.part, s, e1);
        if (prof) {
            CHASE_HIP(hipEventRecord(e2, s));
            prof->push_back(e0);
            prof->push_back(e1);
            prof->push_back(e2);
        }
    }
    finish_degree_one(V, B1, ld, N, n, deg, s);
}

// Same recurrence on complex64 blocks with the complex64 shadow of H: the
// coefficients are formed in FP64 and rounded once to FP32.  Degree-1
// columns end in B1 (the caller converts them back from there).
void filter32_block(const C *Hc, int64_t N, C *V, C *B1, int64_t ld, int n,
                    const int *deg, double mu1, double alpha, double beta,
                    C *fpart, hipStream_t s, std::vector<hipEvent_t> *prof) {
    if (n <= 0) return;
    const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
    const double sigma1 = e / (mu1 - c);
    const double tau = 2.0 / sigma1;
    const int mmax = deg[n - 1];
    auto launch = [&](const C *Y, const C *X, C *W, int cols, double a, double b,
                      double g) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (prof) {
            CHASE_HIP(hipEventCreate(&e0));
            CHASE_HIP(hipEventCreate(&e1));
            CHASE_HIP(hipEventCreate(&e2));
            CHASE_HIP(hipEventRecord(e0, s));
        }
        filter32_gemm(Hc, N, N, Y, ld, X, ld, W, ld, cols, (float)a, (float)b,
                      (float)g, fpart, s, e1);
        if (prof) {
            CHASE_HIP(hipEventRecord(e2, s));
            prof->push_back(e0);
            prof->push_back(e1);
            prof->push_back(e2);
        }
    };
    {
        const double a = sigma1 / e;
        launch(V, nullptr, B1, n, a, -c * a, 0.0);
    }
    double sprev = sigma1;
    int first = 0;
    for (int st = 2; st <= mmax; ++st) {
        const double sigma = 1.0 / (tau - sprev);
        const double a = 2.0 * sigma / e;
        const double g = -sprev * sigma;
        while (first < n && deg[first] < st) ++first;
        const int cols = n - first;
        if (st % 2 == 0) launch(B1 + first, V + first, V + first, cols, a, -c * a, g);
        else launch(V + first, B1 + first, B1 + first, cols, a, -c * a, g);
        sprev = sigma;
    }
}

// ------------------------------------------------------------ QR
// Columns [L, ne) of V: two classical Gram-Schmidt passes against the
// locked columns [0, L), then shifted CholeskyQR3 (Fukaya et al., SIAM J.
// Sci. Comput. 42, 2020) with column scaling; the locked columns are not
// touched.
void qr_block(Z *V, Z *B1, int64_t ld, int64_t N, int L, int ne, Z *G, Z *Bq,
              Z *cwork, Z *gpart, int *dinfo, hipStream_t s) {
    const int n = ne - L;
    if (n <= 0) return;
    Z *Va = V + L;
    if (L > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            gram(V, ld, Va, ld, N, L, n, G, n, gpart, s);
            tsmm(V, ld, G, n, N, L, n, -1.0, Va, ld, 1.0, Va, ld, s);
        }
    }
    Z *cur = Va, *oth = B1 + L;
    for (int pass = 0; pass < 3; ++pass) {
        gram(cur, ld, cur, ld, N, n, n, G, n, gpart, s, true);
        // Shift for the scaled Gram matrix (unit diagonal, so trace = n
        // bounds its 2-norm): 11 (N n + n (n + 1)) u ||G||.
        const double u = 1.1102230246251565e-16;
        const double shift =
            pass == 0 ? 11.0 * ((double)N * n + (double)n * (n + 1)) * u * n : 0.0;
        chol_qr_factor(G, n, shift, Bq, cwork, dinfo + pass, s);
        tsmm(cur, ld, Bq, n, N, n, n, 1.0, nullptr, 0, 0.0, oth, ld, s, true);
        std::swap(cur, oth);
    }
    if (cur != Va) copy_block(cur, ld, Va, ld, N, n, s);
}

// ------------------------------------------------------------ RR + Resid
// Q (N x n, orthonormal): W = H Q, G = Q^H W, G = Y Theta Y^H,
// T = W Y (= H Q Y), Q <- Q Y; resid_j = ||T_j - theta_j (QY)_j||.
void rr_block(const Z *H, int64_t ldh, int64_t N, Z *Q, Z *W, Z *T, Z *B1,
              int64_t ld, int n, Z *G, Z *Y, Z *jwork, double *theta,
              double *resid, Z *fpart, Z *gpart, double *npart, double *hwork,
              hipStream_t s) {
    filter_gemm(H, ldh, N, Q, ld, nullptr, ld, W, ld, n, 1.0, 0.0, 0.0, fpart, s);
    gram(Q, ld, W, ld, N, n, n, G, n, gpart, s);
    hermitise(G, n, s);
    jacobi_eig(G, n, theta, Y, jwork, hwork, s);
    tsmm(W, ld, Y, n, N, n, n, 1.0, nullptr, 0, 0.0, T, ld, s);
    tsmm(Q, ld, Y, n, N, n, n, 1.0, nullptr, 0, 0.0, B1, ld, s);
    if (resid) col_norms(T, ld, B1, ld, theta, N, n, npart, resid, s);
    copy_block(B1, ld, Q, ld, N, n, s);
}

// QR phase inside the solver.  A CholeskyQR breakdown means the filtered
// block is numerically rank deficient (column k depends on columns < k);
// Householder QR would then return a roundoff direction for that column.
// Here the column is replaced by a fresh random vector explicitly and the
// QR is redone from a backup of the block.  Returns the replaced count.
//
// qr_launch enqueues the backup copy, the QR and the copy of its breakdown
// words to the host (then records `done`); qr_finish waits for `done` only
// (work enqueued after the QR, such as the next product, keeps the GPU
// busy meanwhile) and, on a breakdown, redoes the QR from the backup
// synchronously.  Returns true if it had to redo it.
static void qr_launch(Z *V, Z *B1, Z *backup, int64_t ld, int64_t N, int L, int ne, Z *G,
                      Z *Bq, Z *cwork, Z *gpart, int *dinfo, int *hinfo, hipEvent_t done,
                      hipStream_t s) {
    const int n = ne - L;
    if (n <= 0) return;
    copy_block(V + L, ld, backup + L, ld, N, n, s);
    qr_block(V, B1, ld, N, L, ne, G, Bq, cwork, gpart, dinfo, s);
    CHASE_HIP(hipMemcpyAsync(hinfo, dinfo, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    CHASE_HIP(hipEventRecord(done, s));
}

static bool qr_finish(Z *V, Z *B1, Z *backup, int64_t ld, int64_t N, int L, int ne, Z *G,
                      Z *Bq, Z *cwork, Z *gpart, int *dinfo, int *hinfo, hipEvent_t done,
                      uint64_t seed, int &salt, hipStream_t s) {
    const int n = ne - L;
    if (n <= 0) return false;
    CHASE_HIP(hipEventSynchronize(done));
    auto first_bad = [&]() {
        for (int pss = 0; pss < 3; ++pss)
            if (hinfo[pss] != 0) return hinfo[pss] - 1;
        return -1;
    };
    int bad = first_bad();
    if (bad < 0) return false;
    CHASE_HIP(hipStreamSynchronize(s));   // whatever followed the QR is void
    for (int attempt = 0; attempt < n; ++attempt) {
        random_block(backup + L + bad, ld, N, 1, seed, 16u + (uint32_t)salt++, s);
        copy_block(backup + L, ld, V + L, ld, N, n, s);
        qr_block(V, B1, ld, N, L, ne, G, Bq, cwork, gpart, dinfo, s);
        CHASE_HIP(hipMemcpyAsync(hinfo, dinfo, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        CHASE_HIP(hipStreamSynchronize(s));
        bad = first_bad();
        if (bad < 0) return true;
    }
    throw Error(CHASE_EINTERNAL, "QR: repeated CholeskyQR breakdown");
}

namespace {

struct HostBuf {
    double *p = nullptr;
    explicit HostBuf(size_t n) {
        CHASE_HIP(hipHostMalloc((void **)&p, n * sizeof(double), hipHostMallocDefault));
    }
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
};

struct Events {
    std::vector<hipEvent_t> ev;
    hipEvent_t make() {
        hipEvent_t e;
        CHASE_HIP(hipEventCreate(&e));
        ev.push_back(e);
        return e;
    }
    ~Events() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// On an error, waits for the stream before the buffers declared ahead of
// it (pinned host staging in particular) are released: a copy into them may
// still be in flight.
struct SyncOnUnwind {
    hipStream_t s;
    int pending = std::uncaught_exceptions();
    ~SyncOnUnwind() {
        if (std::uncaught_exceptions() > pending) (void)hipStreamSynchronize(s);
    }
};

// Profile events still held when the solve ends early.
struct EventList : std::vector<hipEvent_t> {
    ~EventList() {
        for (auto e : *this) (void)hipEventDestroy(e);
    }
};

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    CHASE_HIP(hipEventElapsedTime(&ms, a, b));
    return 1e-3 * ms;
}

}  // namespace

Result solve(const Problem &p, void *dwork, Z *dV, int64_t ldv, hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    const int64_t N = p.N;
    const chase_opts &o = p.opts;
    const Layout Lo = make_layout(N, p.nev, p.nex, o);
    const int nev = p.nev, ne = Lo.ne;
    char *base = static_cast<char *>(dwork);
    Z *V = reinterpret_cast<Z *>(base + Lo.V);
    Z *B1 = reinterpret_cast<Z *>(base + Lo.B1);
    Z *W = reinterpret_cast<Z *>(base + Lo.W);
    Z *T = reinterpret_cast<Z *>(base + Lo.T);
    Z *fpart = reinterpret_cast<Z *>(base + Lo.fpart);
    Z *gpart = reinterpret_cast<Z *>(base + Lo.gpart);
    Z *G = reinterpret_cast<Z *>(base + Lo.G);
    Z *Bq = reinterpret_cast<Z *>(base + Lo.Bq);
    Z *cwork = reinterpret_cast<Z *>(base + Lo.cwork);
    Z *Y = reinterpret_cast<Z *>(base + Lo.Y);
    Z *jwork = reinterpret_cast<Z *>(base + Lo.jwork);
    double *theta = reinterpret_cast<double *>(base + Lo.theta);
    double *resid = reinterpret_cast<double *>(base + Lo.resid);
    double *npart = reinterpret_cast<double *>(base + Lo.npart);
    int *perm = reinterpret_cast<int *>(base + Lo.perm);
    int *dinfo = reinterpret_cast<int *>(base + Lo.info);
    Z *Lv = reinterpret_cast<Z *>(base + Lo.Lv);
    Z *Lvp = reinterpret_cast<Z *>(base + Lo.Lvp);
    Z *Lw = reinterpret_cast<Z *>(base + Lo.Lw);
    double *Lal = reinterpret_cast<double *>(base + Lo.Lal);
    double *Lbe = reinterpret_cast<double *>(base + Lo.Lbe);
    double *Lpart = reinterpret_cast<double *>(base + Lo.Lpart);
    C *Hc = Lo.mixed ? reinterpret_cast<C *>(base + Lo.Hc) : nullptr;
    C *Vc = Lo.mixed ? reinterpret_cast<C *>(base + Lo.Vc) : nullptr;
    C *Bc = Lo.mixed ? reinterpret_cast<C *>(base + Lo.Bc) : nullptr;
    C *fpart32 = Lo.mixed ? reinterpret_cast<C *>(base + Lo.fpart32) : nullptr;

    const int r = Lo.r, k = Lo.k;
    HostBuf hb((size_t)2 * k * r + 4 * (size_t)ne + 16);
    double *h_al = hb.p, *h_be = hb.p + (size_t)k * r;
    double *h_th = h_be + (size_t)k * r, *h_res = h_th + ne;
    double *h_misc = h_res + ne;   // 3 ints of QR info
    double *h_jac = h_misc + 4;    // 4 Jacobi norms, then its status word
    SyncOnUnwind unwind_sync{s};

    Result R{};
    std::memset(&R.info, 0, sizeof(R.info));
    chase_info &info = R.info;
    Events E;
    JacobiGraphs jgraphs;
    EventList prof, prof32, profx;
    std::vector<int> profx_cols;
    std::vector<hipEvent_t> *profp = o.profile ? &prof : nullptr;
    std::vector<hipEvent_t> *prof32p = o.profile ? &prof32 : nullptr;

    // ---------------- mixed precision: complex64 shadow of H, once per solve
    if (Lo.mixed) {
        hipEvent_t z0 = E.make(), z1 = E.make();
        CHASE_HIP(hipEventRecord(z0, s));
        z2c_matrix(p.H, p.ldh, Hc, N, N, s);
        CHASE_HIP(hipEventRecord(z1, s));
        CHASE_HIP(hipEventSynchronize(z1));
        info.t_shadow = elapsed(z0, z1);
    }
    auto drain_prof = [&]() {
        // Events come in triples around each filter GEMM: before the MFMA
        // kernel, after it (before any split-K reduction), after the step.
        for (size_t i = 0; i + 3 <= prof.size(); i += 3) {
            info.t_filter_kernels += elapsed(prof[i], prof[i + 1]);
            info.filter_launches += 1;
        }
        for (auto e : prof) (void)hipEventDestroy(e);
        prof.clear();
        for (size_t i = 0; i + 3 <= prof32.size(); i += 3) {
            info.t_filter32_kernels += elapsed(prof32[i], prof32[i + 1]);
            info.filter32_launches += 1;
        }
        for (auto e : prof32) (void)hipEventDestroy(e);
        prof32.clear();
        for (size_t i = 0; i + 3 <= profx.size(); i += 3) {
            info.gemm_time += elapsed(profx[i], profx[i + 1]);
            info.gemm_flops += 8.0 * (double)N * (double)N * profx_cols[i / 3];
            info.gemm_launches += 1;
        }
        for (auto e : profx) (void)hipEventDestroy(e);
        profx.clear();
        profx_cols.clear();
    };
    // H times a block outside the filter (Lanczos, Rayleigh-Ritz), timed in
    // profile mode like the filter launches.
    auto gemm_other = [&](const Z *Yb, int64_t ldy, Z *Wb, int64_t ldw, int cols) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (o.profile) {
            CHASE_HIP(hipEventCreate(&e0));
            CHASE_HIP(hipEventCreate(&e1));
            CHASE_HIP(hipEventCreate(&e2));
            CHASE_HIP(hipEventRecord(e0, s));
        }
        filter_gemm(p.H, p.ldh, N, Yb, ldy, nullptr, ldy, Wb, ldw, cols, 1.0, 0.0, 0.0,
                    fpart, s, e1);
        if (o.profile) {
            CHASE_HIP(hipEventRecord(e2, s));
            profx.push_back(e0);
            profx.push_back(e1);
            profx.push_back(e2);
            profx_cols.push_back(cols);
        }
    };

    // ---------------- Lanczos: spectral bounds (once per solve)
    hipEvent_t l0 = E.make(), l1 = E.make();
    CHASE_HIP(hipEventRecord(l0, s));
    random_block(Lw, r, N, r, o.seed, 1u, s);
    lanczos_update(Lv, Lvp, Lw, r, N, r, Lal, Lbe, 0, 1, Lpart, s);
    for (int j = 0; j < k; ++j) {
        gemm_other(Lv, r, Lw, r, r);
        lanczos_update(Lv, Lvp, Lw, r, N, r, Lal, Lbe, j, 0, Lpart, s);
    }
    CHASE_HIP(hipEventRecord(l1, s));
    CHASE_HIP(hipMemcpyAsync(h_al, Lal, sizeof(double) * k * r, hipMemcpyDeviceToHost, s));
    CHASE_HIP(hipMemcpyAsync(h_be, Lbe, sizeof(double) * k * r, hipMemcpyDeviceToHost, s));
    CHASE_HIP(hipStreamSynchronize(s));
    info.t_lanczos = elapsed(l0, l1);
    info.matvecs_total += (int64_t)k * r;
    const double Nd = (double)N;
    info.lanczos_flops = 8.0 * Nd * Nd * r * k;
    info.lanczos_bytes = (double)k * (16.0 * Nd * Nd + 112.0 * Nd * r);
    for (int i = 0; i < k * r; ++i)
        if (!std::isfinite(h_al[i]) || !std::isfinite(h_be[i]))
            throw Error(CHASE_ENONFINITE, "H contains NaN or Inf (seen by Lanczos)");
    const Bounds bd = lanczos_bounds(h_al, h_be, k, r, N, ne);
    info.mu_ne = bd.mu_ne;
    info.beta = bd.bsup;
    info.hnorm_est = bd.hnorm;
    double mu1 = bd.mu1, alpha = bd.mu_ne;
    const double beta = bd.bsup;
    const double tol_abs = p.tol * bd.hnorm;

    // ---------------- start block
    if (o.dV0) {
        const int given = o.v0_cols > 0 ? o.v0_cols : p.nev + p.nex;
        colmajor_to_rowmajor(reinterpret_cast<const Z *>(o.dV0), N, V, ne, N, given, s);
        if (ne > given) random_block(V + given, ne, N, ne - given, o.seed, 2u, s);
    } else {
        random_block(V, ne, N, ne, o.seed, 2u, s);
    }

    const int cap = degree_cap(p.degree_max);
    int d0 = std::min(std::max(2, o.initial_degree), cap);
    d0 += d0 % 2;   // cap is even here unless it is 1
    if (cap == 1) d0 = 1;
    std::vector<int> deg(ne, d0), hperm(ne);
    std::vector<double> lam(ne, 0.0), res(ne, INFINITY);
    // Mixed precision: a column is filtered in FP32 while its residual is
    // above switch_tol * ||H|| and FP32 still improves it (a column whose
    // FP32 iteration gained less than 10x moves to FP64 for good).
    const double sw_abs = o.switch_tol * bd.hnorm;
    std::vector<char> fp32(ne, Lo.mixed ? 1 : 0), use64(ne, 0);
    std::vector<double> res_prev(ne, INFINITY), pred_gain(ne, 1.0);
    std::vector<int> rdeg(ne, d0);           // degrees in Ritz order
    int n32 = Lo.mixed ? ne : 0;             // FP32 columns leading the filter order
    // Residual of each Ritz position at the previous iteration, and the
    // whole-block refinement state (see the stagnation test below).
    std::vector<double> res_last(ne, INFINITY);
    // A warm start begins with a Rayleigh-Ritz of the given block, no
    // filter: its residuals choose the first degrees (converged pairs lock
    // at once) and its largest Ritz value the first damped interval.
    bool refine = o.dV0 != nullptr;
    int last_refine = -100;
    int L = 0;
    int it = 0;
    int qr_salt = 0;
    hipEvent_t ev[6];
    for (auto &e : ev) e = E.make();
    for (it = 1; it <= o.max_iter; ++it) {
        const int n = ne - L;
        CHASE_HIP(hipEventRecord(ev[0], s));
        const double e_half = 0.5 * (beta - alpha);
        // When the search space is the whole space (ne == N) Rayleigh-Ritz
        // is exact and filtering would only make the block ill-conditioned.
        if (!refine && ne < N && e_half > 1e-14 * std::max(1.0, std::fabs(beta))) {
            // Active columns: the FP32 group first, each group by degree.
            if (n32 > 0) {
                info.filter_bytes += (double)deg[L + n32 - 1] * 8.0 * Nd * Nd + 48.0 * Nd * n32;
                for (int j = L; j < L + n32; ++j) info.filter_bytes += 24.0 * Nd * deg[j];
                z2c_block(V + L, ne, Vc, n32, N, n32, s);
                filter32_block(Hc, N, Vc, Bc, n32, n32, deg.data() + L, mu1, alpha,
                               beta, fpart32, s, prof32p);
                const int n1 = degree_one_count(deg.data() + L, n32);
                c2z_block(Bc, n32, V + L, ne, N, n1, s);
                c2z_block(Vc + n1, n32, V + L + n1, ne, N, n32 - n1, s);
                for (int j = L; j < L + n32; ++j) info.matvecs_filter_fp32 += deg[j];
            }
            if (n - n32 > 0) {
                info.filter_bytes += (double)deg[ne - 1] * 16.0 * Nd * Nd;
                for (int j = L + n32; j < ne; ++j) info.filter_bytes += 48.0 * Nd * deg[j];
            }
            if (p.sink) {
                p.sink->run(filter_steps(p.H, p.ldh, N, V + L + n32, B1 + L + n32, ne,
                                         n - n32, deg.data() + L + n32, mu1, alpha, beta,
                                         fpart),
                            s);
                finish_degree_one(V + L + n32, B1 + L + n32, ne, N, n - n32,
                                  deg.data() + L + n32, s);
            } else
                filter_block(p.H, p.ldh, N, V + L + n32, B1 + L + n32, ne, n - n32,
                             deg.data() + L + n32, mu1, alpha, beta, fpart, s, profp);
            for (int j = L; j < ne; ++j) info.matvecs_filter += deg[j];
        }
        CHASE_HIP(hipEventRecord(ev[1], s));
        int *h_qr = reinterpret_cast<int *>(h_misc);
        qr_launch(V, B1, T, ne, N, L, ne, G, Bq, cwork, gpart, dinfo, h_qr, ev[5], s);
        CHASE_HIP(hipEventRecord(ev[2], s));
        Z *Q = V + L;
        // The product W = H Q runs while the host checks the QR.
        gemm_other(Q, ne, W + L, ne, n);
        if (qr_finish(V, B1, T, ne, N, L, ne, G, Bq, cwork, gpart, dinfo, h_qr, ev[5], o.seed,
                      qr_salt, s)) {
            CHASE_HIP(hipEventRecord(ev[2], s));
            gemm_other(Q, ne, W + L, ne, n);
        }
        gram(Q, ne, W + L, ne, N, n, n, G, n, gpart, s);
        hermitise(G, n, s);
        int *h_jst = reinterpret_cast<int *>(h_jac + 4);   // read after the sync below
        jacobi_eig(G, n, theta, Y, jwork, h_jac, s, o.graphs ? &jgraphs : nullptr, h_jst);
        tsmm(Q, ne, Y, n, N, n, n, 1.0, nullptr, 0, 0.0, B1 + L, ne, s);
        CHASE_HIP(hipEventRecord(ev[3], s));
        tsmm(W + L, ne, Y, n, N, n, n, 1.0, nullptr, 0, 0.0, T + L, ne, s);
        col_norms(T + L, ne, B1 + L, ne, theta, N, n, npart, resid, s);
        copy_block(B1 + L, ne, Q, ne, N, n, s);
        CHASE_HIP(hipEventRecord(ev[4], s));
        CHASE_HIP(hipMemcpyAsync(h_th, theta, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        CHASE_HIP(hipMemcpyAsync(h_res, resid, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        CHASE_HIP(hipStreamSynchronize(s));
        jacobi_check_status(n, *h_jst);
        {
            const double nd = n, Ld = L;
            info.qr_flops += 32.0 * Nd * Ld * nd + 48.0 * Nd * nd * nd;
            info.qr_bytes += (L > 0 ? 2.0 * (16.0 * Nd * Ld + 32.0 * Nd * nd) : 0.0) +
                             144.0 * Nd * nd;
            info.rr_flops += 8.0 * Nd * Nd * nd + 16.0 * Nd * nd * nd;
            info.rr_bytes += 16.0 * Nd * Nd + 96.0 * Nd * nd;
            info.resid_flops += 8.0 * Nd * nd * nd + 8.0 * Nd * nd;
            info.resid_bytes += 96.0 * Nd * nd;
        }
        info.t_filter += elapsed(ev[0], ev[1]);
        info.t_qr += elapsed(ev[1], ev[2]);
        info.t_rr += elapsed(ev[2], ev[3]);
        info.t_resid += elapsed(ev[3], ev[4]);
        info.matvecs_total += n;
        if (profp) drain_prof();
        for (int j = 0; j < n; ++j) {
            if (!std::isfinite(h_th[j]) || !std::isfinite(h_res[j]))
                throw Error(CHASE_ENONFINITE, "non-finite Ritz value or residual");
            lam[L + j] = h_th[j];
            res[L + j] = h_res[j];
        }
        if (h_th[n - 1] > beta + 1e-10 * std::max(1.0, bd.hnorm))
            throw Error(CHASE_EBOUNDS, "Ritz value above the spectral upper bound");
        int cnt = 0;
        while (cnt < n && res[L + cnt] <= tol_abs) ++cnt;
        L += cnt;
        info.iterations = it;
        info.nconv = std::min(L, nev);
        info.alpha = alpha;
        info.mu1 = mu1;
        const bool stop = o.on_iteration && o.on_iteration(o.on_iteration_user, &info) != 0;
        if (L >= nev || it == o.max_iter || stop) break;
        // Stagnation just above tol.  A pair locked with a residual just
        // under tol_abs keeps components of its neighbours' eigenvectors
        // (about residual / gap), and every active vector is kept orthogonal
        // to it, so the next vector's residual can stall near tol_abs while
        // the block's span is already accurate.  One Rayleigh-Ritz over the
        // whole block (locked columns included, no filter) splits that span
        // afresh; locking then restarts from the prefix.
        const bool refined_now = refine;
        refine = false;
        if (!refined_now && L > 0 && L < ne && it - last_refine >= 3 &&
            res[L] <= 8.0 * tol_abs && std::isfinite(res_last[L]) &&
            res_last[L] / res[L] < 1.5 && !(Lo.mixed && fp32[L])) {
            refine = true;
            last_refine = it;
            ++info.refinements;
        }
        for (int j = L; j < ne; ++j) res_last[j] = res[j];
        if (refine) {
            for (int j = 0; j < L; ++j) {
                fp32[j] = 0;
                use64[j] = 1;
                res_prev[j] = res[j];
            }
            L = 0;
        }
        // Filter interval, rates and degrees for the next iteration.  The
        // per-vector state is kept in Ritz order (position j = j-th smallest
        // Ritz value of the active block, as Rayleigh-Ritz returns it); only
        // the filter's column order (FP32 group first, then ascending
        // degree) is a permutation of it.
        alpha = h_th[n - 1];
        mu1 = std::min(mu1, h_th[0]);
        const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
        for (int j = L; j < ne; ++j) {
            if (Lo.mixed) {
                // FP32 has stalled on this vector if its residual fell by
                // less than a quarter of the orders of magnitude the filter
                // rate predicted (rho^m), and by less than 8x; it is then
                // filtered in FP64.  Any prediction above 10% counts: near
                // the FP32 floor the target is close, the degree short and
                // rho^m small, and a vector stuck there must still be
                // caught.  The 8x cap keeps the early iterations, whose
                // Ritz values (and so predicted rates) are still rough, from
                // reading a 60x gain against a predicted 1e9 as a stall.
                if (fp32[j] && std::isfinite(res_prev[j]) && pred_gain[j] >= 1.1 &&
                    res_prev[j] / res[j] < std::min(std::pow(pred_gain[j], 0.25), 8.0))
                    use64[j] = 1;
                res_prev[j] = res[j];
                fp32[j] = (!use64[j] && res[j] > sw_abs) ? 1 : 0;
            }
            // FP32 vectors aim at the switch level, FP64 ones at tol.
            const double target = fp32[j] ? std::max(tol_abs, 0.1 * sw_abs) : tol_abs;
            rdeg[j] = degree_for(res[j], target, lam[j], c, e, p.degree_max, o.degree_extra);
            pred_gain[j] = std::pow(rate(lam[j], c, e), (double)rdeg[j]);
        }
        std::vector<int> idx(ne - L);
        std::iota(idx.begin(), idx.end(), L);
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            if (fp32[a] != fp32[b]) return fp32[a] > fp32[b];
            return rdeg[a] < rdeg[b];
        });
        bool ident = true;
        n32 = 0;
        for (int j = 0; j < ne - L; ++j) {
            hperm[j] = idx[j] - L;
            ident = ident && hperm[j] == j;
            deg[L + j] = rdeg[idx[j]];
            n32 += fp32[idx[j]] ? 1 : 0;
        }
        if (!ident) {
            CHASE_HIP(hipMemcpyAsync(perm, hperm.data(), sizeof(int) * (ne - L),
                                     hipMemcpyHostToDevice, s));
            permute_cols(V + L, ne, B1 + L, ne, N, ne - L, perm, s);
            copy_block(B1 + L, ne, V + L, ne, N, ne - L, s);
            // hperm is next written after the next iteration's stream
            // synchronisation, by which time this copy has read it.
        }
    }
    info.alpha = alpha;
    info.mu1 = mu1;
    info.nconv = std::min(L, nev);
    R.status = L >= nev ? CHASE_OK : CHASE_ENOCONV;

    // ---------------- output: the nev lowest, ascending, phase-normalised
    // Columns past nev (out_cols) continue with the rest of the search
    // block, sorted among themselves.
    const int mout = o.out_cols > 0 ? o.out_cols : nev;
    std::vector<int> ord(mout);
    std::iota(ord.begin(), ord.end(), 0);
    auto by_lam = [&](int a, int b) { return lam[a] < lam[b]; };
    std::stable_sort(ord.begin(), ord.begin() + nev, by_lam);
    std::stable_sort(ord.begin() + nev, ord.end(), by_lam);
    R.eigvals.resize(nev);
    R.resid.resize(nev);
    for (int j = 0; j < nev; ++j) {
        R.eigvals[j] = lam[ord[j]];
        R.resid[j] = res[ord[j]];
    }
    CHASE_HIP(hipMemcpyAsync(perm, ord.data(), sizeof(int) * mout, hipMemcpyHostToDevice, s));
    permute_cols(V, ne, B1, mout, N, mout, perm, s);
    phase_normalise_out(B1, mout, N, mout, dV, ldv, npart, s);
    CHASE_HIP(hipStreamSynchronize(s));
    info.filter_flops = 8.0 * (double)N * (double)N * (double)info.matvecs_filter;
    if (o.profile) {
        info.gemm_time += info.t_filter_kernels;
        info.gemm_flops += 8.0 * (double)N * (double)N *
                           (double)(info.matvecs_filter - info.matvecs_filter_fp32);
        info.gemm_launches += info.filter_launches;
    }
    info.matvecs_total += info.matvecs_filter;
    info.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return R;
}

}  // namespace chase
