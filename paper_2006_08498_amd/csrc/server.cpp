// Continuous-batching server: eigenproblems of uneven size are admitted as
// soon as a slot and enough device memory are free, and run concurrently on
// the GPU, one HIP stream per slot.  Each slot holds its problem's H, the
// solver workspace and the eigenvector output resident until the caller
// collects the result.  Admission is first-fit in arrival order against the
// memory budget, so a small request can pass a large one that does not fit
// yet.  A request's result does not depend on what else runs: every kernel
// has a fixed reduction order and each solve uses its own workspace.
#include "../../include/chase_mi355x.h"

#include "common.h"
#include "k_filter_fused.h"
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace chase;

namespace {

using Clock = std::chrono::steady_clock;

enum class St { Queued, Running, Done };

struct Request {
    uint64_t ticket = 0;
    int64_t N = 0;
    int nev = 0, nex = 0, degree_max = 0;
    double tol = 0.0;
    chase_opts opts{};
    // Source of H: a caller device buffer, a host buffer copied at
    // admission, or a fill callback run at admission on the slot's stream.
    const chase_z *dH_user = nullptr;
    std::vector<chase_z> hH;
    chase_fill_fn fill = nullptr;
    void *fill_user = nullptr;
    size_t footprint = 0;   // bytes the server allocates for this request
    St state = St::Queued;
    Clock::time_point t_submit, t_start, t_end;
    // Results (owned until polled).
    int status = CHASE_OK;
    std::string error;
    std::vector<double> eigvals, resid;
    chase_info info{};
    void *dV = nullptr;     // N x nev column-major
    int slot = -1;
    bool collecting = false;   // a poll is copying the result out
};

// Cross-request filter fusion.  Each running solve of a small problem
// (N <= kFuseMaxN) hands the FP64 filter steps of an iteration to the
// server's persistent filter engine
// (FilterEngine, k_filter_fused.hip) instead of launching them: one kernel
// deals out the tiles of every handed-over filter call as soon as each
// call's previous step is complete, so the steps of concurrent solves share
// the GPU with no launch per step and no step boundary between problems.
// The solve's thread waits for its own call only, then goes on with QR on
// its stream.
// Orders up to which a served request's filter calls go to the engine.
constexpr int64_t kFuseMaxN = 8192;

class EngineSink final : public FilterSink {
  public:
    void run(std::vector<FilterCall> &&steps, hipStream_t s) override {
        if (steps.empty()) return;
        // The engine reads the block the work on s produced.
        CHASE_HIP(hipStreamSynchronize(s));
        const int slot = eng_.submit(steps);
        eng_.wait(slot);
        std::lock_guard<std::mutex> lk(m_);
        steps_ += (int64_t)steps.size();
    }
    void stats(int64_t *launches, int64_t *steps) {
        eng_.stats(nullptr, nullptr, launches);
        std::lock_guard<std::mutex> lk(m_);
        *steps = steps_;
    }

  private:
    FilterEngine eng_;
    std::mutex m_;
    int64_t steps_ = 0;
};

}  // namespace

struct chase_server {
    size_t budget = 0;
    int max_slots = 0;
    uint32_t flags = 0;
    double aging_s = 30.0;   // CHASE_SERVER_SHORTEST_FIRST: FIFO after this wait
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    size_t in_use = 0, peak_in_use = 0;
    int running = 0, peak_running = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    hipStream_t copy_stream = nullptr;   // poll's result copies (non-blocking)
    std::mutex copy_mu;
    int device = 0;
    std::unique_ptr<EngineSink> broker;   // CHASE_SERVER_FUSE_FILTER
};

namespace {

double secs(Clock::duration d) { return std::chrono::duration<double>(d).count(); }

size_t footprint(const Request &r) {
    const size_t ws = make_layout(r.N, r.nev, r.nex, r.opts).total;
    const size_t hb = r.dH_user ? 0 : (size_t)r.N * r.N * sizeof(Z);
    return ws + hb + (size_t)r.N * r.nev * sizeof(Z) + 3 * 256;
}

// Estimated work of a request: the filter's N^2 per column times the
// subspace size (the per-request iteration count is not known up front).
double est_work(const Request &r) {
    return (double)r.N * (double)r.N * (double)(r.nev + r.nex);
}

// The next request to admit among those that fit the free memory: the
// first in arrival order, or (CHASE_SERVER_SHORTEST_FIRST) the one with the
// least estimated work, except that a request waiting longer than aging_s
// goes first (in arrival order) so that large requests are not starved.
Request *pick(chase_server *s) {
    auto fits = [&](const Request *r) { return r->footprint + s->in_use <= s->budget; };
    auto take = [&](std::deque<Request *>::iterator it) {
        Request *r = *it;
        s->pending.erase(it);
        return r;
    };
    if (!(s->flags & CHASE_SERVER_SHORTEST_FIRST)) {
        for (auto it = s->pending.begin(); it != s->pending.end(); ++it)
            if (fits(*it)) return take(it);
        return nullptr;
    }
    const auto now = Clock::now();
    auto best = s->pending.end();
    for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
        if (!fits(*it)) continue;
        if (secs(now - (*it)->t_submit) > s->aging_s) return take(it);
        if (best == s->pending.end() || est_work(**it) < est_work(**best)) best = it;
    }
    return best == s->pending.end() ? nullptr : take(best);
}

void run_one(chase_server *s, Request *r, int slot) {
    hipStream_t st = s->streams[slot];
    void *dH = nullptr, *dW = nullptr, *dV = nullptr;
    try {
        const Layout lay = make_layout(r->N, r->nev, r->nex, r->opts);
        CHASE_HIP(hipMalloc(&dW, lay.total));
        CHASE_HIP(hipMalloc(&dV, (size_t)r->N * r->nev * sizeof(Z)));
        const Z *H = reinterpret_cast<const Z *>(r->dH_user);
        if (!H) {
            CHASE_HIP(hipMalloc(&dH, (size_t)r->N * r->N * sizeof(Z)));
            if (r->fill) {
                const int fst = r->fill(reinterpret_cast<chase_z *>(dH), r->N, r->N,
                                        r->fill_user, st);
                if (fst != 0) throw Error(CHASE_EINVAL, "fill callback failed");
            } else {
                CHASE_HIP(hipMemcpyAsync(dH, r->hH.data(), r->hH.size() * sizeof(Z),
                                         hipMemcpyHostToDevice, st));
                CHASE_HIP(hipStreamSynchronize(st));
                std::vector<chase_z>().swap(r->hH);
            }
            H = reinterpret_cast<const Z *>(dH);
        }
        // Small problems (whose own filter launches underfill the GPU) hand
        // their filter calls to the persistent engine; large ones launch
        // their own, which fill the GPU alone.
        FilterSink *sink = r->N <= kFuseMaxN ? s->broker.get() : nullptr;
        Problem p{H, r->N, r->N, r->nev, r->nex, r->tol, r->degree_max, r->opts, sink};
        Result R = solve(p, dW, reinterpret_cast<Z *>(dV), r->N, st);
        r->eigvals = std::move(R.eigvals);
        r->resid = std::move(R.resid);
        r->info = R.info;
        r->status = R.status;
        if (R.status == CHASE_ENOCONV) r->error = "not converged after max_iter iterations";
    } catch (const Error &e) {
        r->status = e.status;
        r->error = e.what();
    } catch (const std::exception &e) {
        r->status = CHASE_EINTERNAL;
        r->error = e.what();
    }
    (void)hipStreamSynchronize(st);
    if (dW) (void)hipFree(dW);
    if (dH) (void)hipFree(dH);
    if (r->status != CHASE_OK && r->status != CHASE_ENOCONV && dV) {
        (void)hipFree(dV);
        dV = nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    r->dV = dV;
    r->t_end = Clock::now();
    r->state = St::Done;
    // Workspace and H are released now; the eigenvectors stay counted until
    // the caller polls them.
    const size_t keep = dV ? (size_t)r->N * r->nev * sizeof(Z) + 256 : 0;
    s->in_use -= r->footprint - keep;
    r->footprint = keep;
    --s->running;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
}

void worker(chase_server *s, int slot) {
    (void)hipSetDevice(s->device);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || (r = pick(s)) != nullptr; });
            if (!r) return;   // stop
            r->state = St::Running;
            r->slot = slot;
            r->t_start = Clock::now();
            s->in_use += r->footprint;
            s->peak_in_use = std::max(s->peak_in_use, s->in_use);
            ++s->running;
            s->peak_running = std::max(s->peak_running, s->running);
        }
        run_one(s, r, slot);
    }
}

thread_local std::string g_srv_err;

int srv_fail(int st, const std::string &m) {
    g_srv_err = m;
    return st;
}

int submit_common(chase_server *s, std::unique_ptr<Request> r, uint64_t *ticket) {
    if (!s || !ticket) return srv_fail(CHASE_EINVAL, "NULL server or ticket");
    try {
        validate_problem(r->N, r->nev, r->nex, r->tol, r->degree_max, r->opts);
    } catch (const Error &e) {
        return srv_fail(e.status, e.what());
    }
    if (r->opts.dV0 || r->opts.v0_cols != 0)
        return srv_fail(CHASE_EINVAL, "warm start is not supported by the server");
    if (r->opts.out_cols != 0 && r->opts.out_cols != r->nev)
        return srv_fail(CHASE_EINVAL, "the server returns nev columns (out_cols must be 0)");
    r->footprint = footprint(*r);
    if (r->footprint > s->budget)
        return srv_fail(CHASE_ENOMEM, "request footprint " + std::to_string(r->footprint) +
                                          " exceeds the server budget");
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->cv_work.notify_all();
    return CHASE_OK;
}

}  // namespace

extern "C" {

chase_server *chase_server_create(size_t hbm_budget_bytes, int32_t max_slots, uint32_t flags) {
    try {
        if (max_slots < 1 || max_slots > 64) {
            g_srv_err = "max_slots must be in [1, 64]";
            return nullptr;
        }
        if (flags & ~(uint32_t)(CHASE_SERVER_FUSE_FILTER | CHASE_SERVER_SHORTEST_FIRST)) {
            g_srv_err = "unknown server flags";
            return nullptr;
        }
        auto *s = new chase_server();
        CHASE_HIP(hipGetDevice(&s->device));
        if (hbm_budget_bytes == 0) {
            size_t fr = 0, tot = 0;
            CHASE_HIP(hipMemGetInfo(&fr, &tot));
            const size_t reserve = std::min<size_t>(fr / 10, (size_t)8 << 30);
            hbm_budget_bytes = fr - reserve;
        }
        s->budget = hbm_budget_bytes;
        s->max_slots = max_slots;
        s->flags = flags;
        for (int i = 0; i < max_slots; ++i) {
            hipStream_t st;
            CHASE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            s->streams.push_back(st);
        }
        CHASE_HIP(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
        if (flags & CHASE_SERVER_FUSE_FILTER) s->broker = std::make_unique<EngineSink>();
        for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker, s, i);
        return s;
    } catch (const std::exception &e) {
        g_srv_err = e.what();
        return nullptr;
    }
}

int chase_server_submit(chase_server *s, const chase_z *H, int is_device, int64_t N,
                        int64_t ldh, int32_t nev, int32_t nex, double tol,
                        int32_t degree_max, const chase_opts *o, uint64_t *ticket) {
    try {
        if (!H) return srv_fail(CHASE_EINVAL, "H is NULL");
        if (ldh < N) return srv_fail(CHASE_EINVAL, "ldh < N");
        auto r = std::make_unique<Request>();
        r->N = N;
        r->nev = nev;
        r->nex = nex;
        r->tol = tol;
        r->degree_max = degree_max;
        chase_default_opts(&r->opts);
        if (o) r->opts = *o;
        if (is_device) {
            if (ldh != N) return srv_fail(CHASE_EINVAL, "device H must have ldh == N");
            r->dH_user = H;
        } else {
            r->hH.resize((size_t)N * N);
            for (int64_t j = 0; j < N; ++j)
                std::memcpy(&r->hH[(size_t)j * N], H + (size_t)j * ldh, sizeof(chase_z) * N);
        }
        return submit_common(s, std::move(r), ticket);
    } catch (const std::bad_alloc &) {
        return srv_fail(CHASE_ENOMEM, "host allocation failed");
    }
}

int chase_server_submit_fill(chase_server *s, chase_fill_fn fill, void *user, int64_t N,
                             int32_t nev, int32_t nex, double tol, int32_t degree_max,
                             const chase_opts *o, uint64_t *ticket) {
    if (!fill) return srv_fail(CHASE_EINVAL, "fill is NULL");
    auto r = std::make_unique<Request>();
    r->N = N;
    r->nev = nev;
    r->nex = nex;
    r->tol = tol;
    r->degree_max = degree_max;
    chase_default_opts(&r->opts);
    if (o) r->opts = *o;
    r->fill = fill;
    r->fill_user = user;
    return submit_common(s, std::move(r), ticket);
}

int chase_server_poll(chase_server *s, uint64_t ticket, double *h_eigvals,
                      double *h_resid, chase_z *dV, int64_t ldv,
                      chase_info *info, double *h_times3) {
    if (!s) return srv_fail(CHASE_EINVAL, "NULL server");
    Request *r = nullptr;
    {
        // Claim the result under the lock: a second poll of the same ticket
        // while this one copies it out sees it claimed and is refused.
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return srv_fail(CHASE_EINVAL, "unknown ticket");
        r = it->second.get();
        if (r->state != St::Done) return CHASE_PENDING;
        if (r->collecting) return srv_fail(CHASE_EINVAL, "the result is being collected");
        if (r->dV && (!dV || ldv < r->N)) return srv_fail(CHASE_EINVAL, "dV is NULL or ldv < N");
        r->collecting = true;
    }
    int st = r->status;
    try {
        if (r->dV) {
            std::lock_guard<std::mutex> lk(s->copy_mu);
            CHASE_HIP(hipMemcpy2DAsync(dV, (size_t)ldv * sizeof(Z), r->dV,
                                       (size_t)r->N * sizeof(Z), (size_t)r->N * sizeof(Z),
                                       r->nev, hipMemcpyDeviceToDevice, s->copy_stream));
            CHASE_HIP(hipStreamSynchronize(s->copy_stream));
        }
        if (h_eigvals && !r->eigvals.empty())
            std::copy(r->eigvals.begin(), r->eigvals.end(), h_eigvals);
        if (h_resid && !r->resid.empty()) std::copy(r->resid.begin(), r->resid.end(), h_resid);
        if (info) *info = r->info;
        if (h_times3) {
            h_times3[0] = secs(r->t_start - r->t_submit);   // queue wait
            h_times3[1] = secs(r->t_end - r->t_start);      // on the GPU
            h_times3[2] = secs(r->t_end - r->t_submit);     // latency
        }
    } catch (const Error &e) {
        std::lock_guard<std::mutex> lk(s->mu);
        r->collecting = false;   // the result stays; the caller may poll again
        return srv_fail(e.status, e.what());
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->dV) (void)hipFree(r->dV);
    s->in_use -= r->footprint;
    if (st != CHASE_OK) g_srv_err = r->error;
    s->reqs.erase(ticket);
    s->cv_work.notify_all();
    return st;
}

int chase_server_wait(chase_server *s, uint64_t ticket, double timeout_s) {
    if (!s) return srv_fail(CHASE_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto done = [&] {
        auto it = s->reqs.find(ticket);
        return it == s->reqs.end() || it->second->state == St::Done;
    };
    if (timeout_s < 0) s->cv_done.wait(lk, done);
    else s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done);
    return done() ? CHASE_OK : CHASE_PENDING;
}

int chase_server_set_aging(chase_server *s, double seconds) {
    if (!s || !(seconds >= 0.0)) return srv_fail(CHASE_EINVAL, "NULL server or negative aging");
    std::lock_guard<std::mutex> lk(s->mu);
    s->aging_s = seconds;
    s->cv_work.notify_all();
    return CHASE_OK;
}

int chase_server_fusion_stats(chase_server *s, int64_t *ticks, int64_t *steps) {
    if (!s || !ticks || !steps) return srv_fail(CHASE_EINVAL, "NULL argument");
    *ticks = *steps = 0;
    if (s->broker) s->broker->stats(ticks, steps);
    return CHASE_OK;
}

int chase_server_stats(chase_server *s, size_t *bytes_in_use, size_t *peak_bytes,
                       int32_t *running, int32_t *peak_running, int32_t *queued) {
    if (!s) return srv_fail(CHASE_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (bytes_in_use) *bytes_in_use = s->in_use;
    if (peak_bytes) *peak_bytes = s->peak_in_use;
    if (running) *running = s->running;
    if (peak_running) *peak_running = s->peak_running;
    if (queued) *queued = (int32_t)s->pending.size();
    return CHASE_OK;
}

const char *chase_server_last_error(void) { return g_srv_err.c_str(); }

void chase_server_destroy(chase_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->pending.clear();
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    s->broker.reset();
    for (auto &kv : s->reqs)
        if (kv.second->dV) (void)hipFree(kv.second->dV);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
}

}  // extern "C"
