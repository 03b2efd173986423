// Persistent filter engine (the serving form of the Filter phase): one
// long-lived kernel runs the recurrence steps of the filter calls (jobs) of
// every eigenproblem that hands it one, whenever they arrive, the steps of
// different jobs interleaved freely on the GPU and the steps of one job
// kept in order on the device, so no launch boundary, host round trip or
// grid tail separates one step from the next or one problem from another.
//
// Work description.  A job's filter call is a chain of stages: one stage
// per recurrence step and column piece (filter_steps / filter_pieces), in
// the order filter_gemm would run them alone.  A stage is a set of items:
// the MFMA tiles of its plan (64 rows x up to 16*kFW columns of one K range)
// and, when its plan splits K, one reduction per 64-row block, which waits
// for the stage's tiles.  Each XCD deals out the items of its own row blocks
// (row block rb on XCD rb % 8, as a launch of its own places it, so a row
// panel of H is shared through that XCD's L2; workgroup ids are dealt
// round-robin to the XCDs).
//
// Scheduling.  A workgroup scans the active jobs, takes the next item of a
// job's current stage from its XCD's share (an atomic ticket), runs it and
// counts it done; the workgroup that completes a stage moves the job to the
// next one, and completing the last stage marks the job done for the host.
// A workgroup never waits for another: it only takes items whose
// dependencies are complete, so the engine cannot deadlock, and idle
// workgroups poll (with sleeps) for new jobs or the host's stop word.
//
// Results.  Each output column is computed with the K ranges, split count,
// MFMA order, reduction order and explicitly fused epilogue of filter_gemm
// alone (only the number of 16-column tiles one wave carries differs, which
// no column's arithmetic depends on), so a job's result is bitwise the one
// the job gives alone.
//
// Memory ordering.  Items of one stage run on every XCD and each XCD has its
// own L2: a finished item is published with an agent-scope release (L2
// write-back) before its counters move, and a workgroup does an acquire
// (L2 invalidate) the first time it works on a job's stage.  The host
// publishes a job in host-coherent memory after its descriptors reached the
// device (system-scope acquire on the kernel's side), and the kernel marks it
// done there after a system-scope release.
#include "k_filter_fused.h"

#include "k_filter_kern.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

namespace chase {

// One stage: one recurrence step of one job over one column piece.
struct EngStage {
    filter_detail::FilterArgs A;
    int wn;          // tile width of the piece's plan (16-column tiles)
    int sub;         // sub-tiles per plan tile: ceil(wn / kFW)
    int tiles;       // rb * cb * splits * sub, on all XCDs
    int reduces;     // rb when the plan splits K, else 0
    int ntile[8];    // tiles of each XCD's row blocks
    int nred[8];     // reductions of each XCD's row blocks
};
// Per-stage counters: tickets dealt per XCD (tiles, reductions), tiles done,
// items done.
struct EngCounters {
    int tick[8], rtick[8], tiles_done, all_done, pad[14];
};
static_assert(sizeof(EngCounters) == 128, "one counter block per 128 bytes");

// Host-coherent control block (pinned host memory the GPU reads and writes
// with system-scope atomics).
struct EngCtl {
    int stop;                       // host: 1 = leave when idle
    int err;                        // kernel: a job could not be run
    unsigned long long active;      // host: bit j = job slot j is running
    int done[kEngineSlots];         // kernel: 1 when slot j's job finished
    int gen[kEngineSlots];          // host: submission counter of slot j
};

// Device-side slot table.
struct EngSlot {
    int nstages, cur, gen, pad;
};

namespace {

using namespace filter_detail;

// Tile width (16-column MFMA tiles per wave) of the persistent kernel; a
// plan tile of width wn runs as ceil(wn / kFW) sub-tiles.
constexpr int kFW = 5;

__device__ __forceinline__ int load_acquire_agent(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Columns [col0, col0 + 16*aw) of row block rb over K range sp of stage A:
// filter_tile's arithmetic with a run-time number aw <= kFW of 16-column
// tiles.
__device__ __forceinline__ void fused_tile(const FilterArgs &A, int rb, int sp, int col0,
                                           int aw) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int N = A.N, n = A.n;
    const int row0 = rb * 64 + wave * 16;
    if (row0 >= N) return;
    const int kbeg = sp * A.kchunk;
    const int kend = max(kbeg, min(N, kbeg + A.kchunk));
    const int arow = min(row0 + r, N - 1);
    const Z *hp = A.H + arow + (int64_t)(kbeg + q) * A.ldh;
    const int64_t hstep = 4 * A.ldh;
    int ycol[kFW];
#pragma unroll
    for (int c = 0; c < kFW; ++c) ycol[c] = min(col0 + 16 * c + r, n - 1);
    const Z *yp = A.Y + (int64_t)(kbeg + q) * A.ldy;
    const int64_t ystep = 4 * A.ldy;

    v4d cr[kFW], ci[kFW];
#pragma unroll
    for (int c = 0; c < kFW; ++c) {
        cr[c] = v4d{0.0, 0.0, 0.0, 0.0};
        ci[c] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    // The same four MFMAs per complex product, in the same order per
    // accumulator, as filter_tile (tiles c >= aw are skipped).
#define FUSED_KSTEP(hv, yv)                                                   \
    {                                                                         \
        const double nhy_ = -(hv).y;                                          \
        _Pragma("unroll") for (int c = 0; c < kFW; ++c) if (c < aw)           \
            cr[c] = mfma64((hv).x, (yv)[c].x, cr[c]);                         \
        _Pragma("unroll") for (int c = 0; c < kFW; ++c) if (c < aw)           \
            ci[c] = mfma64((hv).x, (yv)[c].y, ci[c]);                         \
        _Pragma("unroll") for (int c = 0; c < kFW; ++c) if (c < aw)           \
            cr[c] = mfma64(nhy_, (yv)[c].y, cr[c]);                           \
        _Pragma("unroll") for (int c = 0; c < kFW; ++c) if (c < aw)           \
            ci[c] = mfma64((hv).y, (yv)[c].x, ci[c]);                         \
    }
    const int nsteps = (kend - kbeg) >> 2;
    if (nsteps > 0) {
        Z h = *hp;
        Z y[kFW];
#pragma unroll
        for (int c = 0; c < kFW; ++c) y[c] = c < aw ? yp[ycol[c]] : Z{0.0, 0.0};
        for (int st = 0; st + 1 < nsteps; ++st) {
            const Z *hn_p = hp + (int64_t)(st + 1) * hstep;
            const Z *yn_p = yp + (int64_t)(st + 1) * ystep;
            const Z hn = *hn_p;
            Z yn[kFW];
#pragma unroll
            for (int c = 0; c < kFW; ++c) yn[c] = c < aw ? yn_p[ycol[c]] : Z{0.0, 0.0};
            FUSED_KSTEP(h, y);
            h = hn;
#pragma unroll
            for (int c = 0; c < kFW; ++c) y[c] = yn[c];
        }
        FUSED_KSTEP(h, y);
    }
    const int k = kbeg + 4 * nsteps;
    if (k < kend) {
        const bool ok = (k + q) < kend;
        const Z *hq = hp + (int64_t)nsteps * hstep;
        const Z *yq = yp + (int64_t)nsteps * ystep;
        const Z h = ok ? *hq : Z{0.0, 0.0};
        Z y[kFW];
#pragma unroll
        for (int c = 0; c < kFW; ++c) y[c] = (ok && c < aw) ? yq[ycol[c]] : Z{0.0, 0.0};
        FUSED_KSTEP(h, y);
    }
#undef FUSED_KSTEP
#pragma unroll
    for (int c = 0; c < kFW; ++c) {
        if (c >= aw) continue;
        const int col = col0 + 16 * c + r;
        if (col >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + q + 4 * v;
            if (row >= N) continue;
            const double sr = cr[c][v], si = ci[c][v];
            if (A.splits == 1) {
                const Z yv = A.Y[(int64_t)row * A.ldy + col];
                const Z xv = A.g != 0.0 ? A.X[(int64_t)row * A.ldx + col] : Z{0.0, 0.0};
                A.W[(int64_t)row * A.ldw + col] = filter_epilogue(sr, si, yv, xv, A.a, A.b, A.g);
            } else {
                A.part[((int64_t)sp * N + row) * n + col] = Z{sr, si};
            }
        }
    }
}

// Ordered sum of the split-K partials of rows [64 rb, 64 rb + 64) plus the
// epilogue, exactly as k_filter_reduce does for each entry.
__device__ __forceinline__ void fused_reduce(const FilterArgs &A, int rb) {
    const int N = A.N, n = A.n;
    const int r0 = rb * 64, r1 = min(N, r0 + 64);
    const int64_t total = (int64_t)N * n;
    for (int64_t e = (int64_t)r0 * n + threadIdx.x; e < (int64_t)r1 * n; e += blockDim.x) {
        const int64_t row = e / n;
        const int col = (int)(e - row * n);
        double sr = 0.0, si = 0.0;
        for (int s = 0; s < A.splits; ++s) {
            const Z p = A.part[(int64_t)s * total + e];
            sr += p.x;
            si += p.y;
        }
        const Z yv = A.Y[row * A.ldy + col];
        const Z xv = A.g != 0.0 ? A.X[row * A.ldx + col] : Z{0.0, 0.0};
        A.W[row * A.ldw + col] = filter_epilogue(sr, si, yv, xv, A.a, A.b, A.g);
    }
}

__device__ __forceinline__ int ld_sys(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned long long ld_sys64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ int ld_agent(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Idle scans (each a sleep of 16 * 64 cycles and a pass over the active
// slots, with a host read every kHostReadEvery scans: about half a
// microsecond to a microsecond) after which a workgroup leaves even without
// the stop word, a backstop if the host never sets it: about 10 s.
constexpr int kIdleLimit = 12 << 20;

// Scans between reads of the host's control words (each a PCIe read):
// a new job or the stop word is seen within about that many scans.
constexpr int kHostReadEvery = 64;

__global__ __launch_bounds__(256) void k_filter_engine(EngCtl *ctl, EngSlot *slots,
                                                       const EngStage *__restrict__ stages,
                                                       EngCounters *cnt, int max_stages) {
    __shared__ int sh_job, sh_stage, sh_item, sh_stop;
    // Per workgroup: the host's active mask and slot generations as last
    // read, and the (generation, stage) of each slot it last acquired for,
    // so it invalidates its caches once per stage it joins.
    __shared__ int gen_host[kEngineSlots], seen_gen[kEngineSlots], seen_stage[kEngineSlots];
    __shared__ unsigned long long act_cache;
    __shared__ int since_read;
    const int xcd = blockIdx.x & 7;
    const int t = threadIdx.x;
    for (int j = t; j < kEngineSlots; j += blockDim.x) {
        seen_gen[j] = -1;
        seen_stage[j] = -1;
        gen_host[j] = -1;
    }
    if (t == 0) {
        act_cache = 0ull;
        since_read = kHostReadEvery;   // read the host words first
    }
    int idle = 0;
    int rot = (blockIdx.x >> 3) % kEngineSlots;
    for (;;) {
        if (t == 0) {
            sh_job = -1;
            sh_stop = 0;
            if (since_read >= kHostReadEvery) {
                since_read = 0;
                const unsigned long long act = ld_sys64(&ctl->active);
                for (int j = 0; j < kEngineSlots; ++j)
                    if ((act >> j) & 1ull) gen_host[j] = ld_sys(&ctl->gen[j]);
                sh_stop = ld_sys(&ctl->stop);
                // The host published these jobs after their descriptors
                // reached device memory.
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");   // system scope
                act_cache = act;
            }
            const unsigned long long act = act_cache;
            for (int k = 0; k < kEngineSlots && act != 0ull && sh_job < 0; ++k) {
                const int j = (rot + k) % kEngineSlots;
                if (!((act >> j) & 1ull)) continue;
                EngSlot *sl = slots + j;
                // The device record must be the one the host published (a
                // slot being refilled for its next job is skipped).
                const int g = ld_agent(&sl->gen);
                if (g != gen_host[j]) continue;
                const int ns = ld_agent(&sl->nstages);
                const int c = ld_agent(&sl->cur);
                if (c >= ns) continue;   // finished
                const int si = j * max_stages + c;
                if (seen_gen[j] != g || seen_stage[j] != c) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    seen_gen[j] = g;
                    seen_stage[j] = c;
                }
                const EngStage &S = stages[si];
                EngCounters *C = cnt + si;
                if (ld_agent(&C->tiles_done) < S.tiles) {
                    if (ld_agent(&C->tick[xcd]) >= S.ntile[xcd]) continue;
                    const int tk = atomicAdd(&C->tick[xcd], 1);
                    if (tk >= S.ntile[xcd]) continue;
                    sh_job = j;
                    sh_stage = si;
                    sh_item = tk;
                } else {
                    if (ld_agent(&C->rtick[xcd]) >= S.nred[xcd]) continue;
                    const int tk = atomicAdd(&C->rtick[xcd], 1);
                    if (tk >= S.nred[xcd]) continue;
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the tiles' partials
                    sh_job = j;
                    sh_stage = si;
                    sh_item = S.tiles + tk;
                }
            }
            ++since_read;
        }
        __syncthreads();
        const int job = sh_job;
        if (job < 0) {
            if (sh_stop || ++idle > kIdleLimit) return;   // uniform: read after the barrier
            rot = (rot + 1) % kEngineSlots;
            __builtin_amdgcn_s_sleep(16);
            continue;
        }
        idle = 0;
        const int si = sh_stage, item = sh_item;
        const EngStage &S = stages[si];
        if (item < S.tiles) {
            // item = ((rb_local * splits + sp) * cb + cb_i) * sub + s over
            // this XCD's row blocks (rb = 8 rb_local + xcd).
            int x = item;
            const int s = x % S.sub;
            x /= S.sub;
            const int cbi = x % S.A.cb_count;
            x /= S.A.cb_count;
            const int sp = x % S.A.splits;
            const int rb = (x / S.A.splits) * 8 + xcd;
            const int t0 = s * kFW;
            fused_tile(S.A, rb, sp, cbi * 16 * S.wn + 16 * t0, min(kFW, S.wn - t0));
        } else {
            fused_reduce(S.A, (item - S.tiles) * 8 + xcd);
        }
        __syncthreads();   // every store of the item issued and complete
        if (t == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            EngCounters *C = cnt + si;
            if (item < S.tiles) atomicAdd(&C->tiles_done, 1);
            const int total = S.tiles + S.reduces;
            if (atomicAdd(&C->all_done, 1) + 1 == total) {
                // This workgroup finished the stage: having seen every other
                // item's count, it publishes them all with the move to the
                // next stage.
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                EngSlot *sl = slots + job;
                const int nxt = ld_agent(&sl->cur) + 1;
                __hip_atomic_store(&sl->cur, nxt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (nxt >= ld_agent(&sl->nstages)) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");   // system scope
                    __hip_atomic_store(&ctl->done[job], 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
        }
        rot = (rot + 1) % kEngineSlots;
    }
}

}  // namespace

int fused_tile_width() { return kFW; }

FilterEngine::FilterEngine() {
    CHASE_HIP(hipGetDevice(&device_));
    CHASE_HIP(hipStreamCreateWithFlags(&ks_, hipStreamNonBlocking));
    CHASE_HIP(hipStreamCreateWithFlags(&cs_, hipStreamNonBlocking));
    CHASE_HIP(hipEventCreateWithFlags(&kdone_, hipEventDisableTiming));
    CHASE_HIP(hipHostMalloc(&ctl_, sizeof(EngCtl), hipHostMallocCoherent));
    std::memset(ctl_, 0, sizeof(EngCtl));
    max_stages_ = kEngineMaxStages;
    const size_t nst = (size_t)kEngineSlots * max_stages_;
    CHASE_HIP(hipMalloc(&dslots_, sizeof(EngSlot) * kEngineSlots));
    CHASE_HIP(hipMalloc(&dstages_, sizeof(EngStage) * nst));
    CHASE_HIP(hipMalloc(&dcnt_, sizeof(EngCounters) * nst));
    CHASE_HIP(hipMemset(dslots_, 0, sizeof(EngSlot) * kEngineSlots));
    CHASE_HIP(hipMemset(dcnt_, 0, sizeof(EngCounters) * nst));
    stage_bytes_ = sizeof(EngStage) * max_stages_;
    const size_t staging = stage_bytes_ + sizeof(EngCounters) * max_stages_ + sizeof(EngSlot);
    for (int j = 0; j < kEngineSlots; ++j)
        CHASE_HIP(hipHostMalloc(&hstage_[j], staging, hipHostMallocDefault));
    int per_cu = 0;
    CHASE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_filter_engine, 256, 0));
    int cus = 0;
    CHASE_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device_));
    // One workgroup per CU: the engine stays resident while jobs are in
    // flight, so it keeps to a quarter of each CU's waves and under half of
    // its registers, leaving room for the other kernels of the same solves.
    grid_ = std::max(8, std::min(std::max(1, per_cu), 1) * cus);
    grid_ = (grid_ + 7) / 8 * 8;   // whole rounds over the XCDs
}

FilterEngine::~FilterEngine() {
    try {
        std::lock_guard<std::mutex> lk(mu_);
        stop_kernel_locked();
    } catch (...) {
    }
    for (auto p : hstage_)
        if (p) (void)hipHostFree(p);
    if (dcnt_) (void)hipFree(dcnt_);
    if (dstages_) (void)hipFree(dstages_);
    if (dslots_) (void)hipFree(dslots_);
    if (ctl_) (void)hipHostFree(ctl_);
    if (kdone_) (void)hipEventDestroy(kdone_);
    if (cs_) (void)hipStreamDestroy(cs_);
    if (ks_) (void)hipStreamDestroy(ks_);
}

static std::vector<EngStage> build_stages(const std::vector<FilterCall> &steps) {
    std::vector<EngStage> st;
    for (const FilterCall &f : steps) {
        if (f.n <= 0 || f.N <= 0) continue;
        for (const FilterPiece &pc : filter_pieces(f.N, f.n)) {
            FilterCall c = f;
            c.Y += pc.c0;
            if (c.X) c.X += pc.c0;
            c.W += pc.c0;
            c.n = pc.n;
            if (pc.p.splits > 1 && !c.part) throw Error(7, "filter engine: missing partials");
            EngStage S{};
            S.A = filter_args(pc.p, c);
            S.wn = pc.p.wn;
            S.sub = (pc.p.wn + kFW - 1) / kFW;
            S.tiles = pc.p.rb * pc.p.cb * pc.p.splits * S.sub;
            S.reduces = pc.p.splits > 1 ? pc.p.rb : 0;
            const int per_rb = pc.p.splits * pc.p.cb * S.sub;
            for (int x = 0; x < 8; ++x) {
                const int rbs = pc.p.rb > x ? (pc.p.rb - x + 7) / 8 : 0;
                S.ntile[x] = rbs * per_rb;
                S.nred[x] = S.reduces ? rbs : 0;
            }
            st.push_back(S);
        }
    }
    return st;
}

void FilterEngine::launch_locked() {
    ctl_->stop = 0;
    hipLaunchKernelGGL(k_filter_engine, dim3(grid_), dim3(256), 0, ks_, ctl_, dslots_, dstages_,
                       dcnt_, max_stages_);
    check_launch("k_filter_engine");
    CHASE_HIP(hipEventRecord(kdone_, ks_));
    running_ = true;
    ++launches_;
}

bool FilterEngine::kernel_exited_locked() {
    if (!running_) return true;
    const hipError_t q = hipEventQuery(kdone_);
    if (q == hipErrorNotReady) return false;
    CHASE_HIP(q);
    running_ = false;
    return true;
}

void FilterEngine::stop_kernel_locked() {
    if (!running_) return;
    __atomic_store_n(&ctl_->stop, 1, __ATOMIC_SEQ_CST);
    CHASE_HIP(hipEventSynchronize(kdone_));
    running_ = false;
    __atomic_store_n(&ctl_->stop, 0, __ATOMIC_SEQ_CST);
}

int FilterEngine::submit(const std::vector<FilterCall> &steps) {
    const std::vector<EngStage> st = build_stages(steps);
    if ((int)st.size() > max_stages_)
        throw Error(1, "filter engine: more than " + std::to_string(max_stages_) + " stages");
    std::unique_lock<std::mutex> lk(mu_);
    int slot = -1;
    cv_.wait(lk, [&] {
        for (int j = 0; j < kEngineSlots; ++j)
            if (!busy_[j]) {
                slot = j;
                return true;
            }
        return false;
    });
    busy_[slot] = true;
    ++active_;
    const int g = ++gen_[slot];
    ctl_->done[slot] = 0;
    if (st.empty()) {
        ctl_->done[slot] = 1;
        return slot;
    }
    // Descriptors, zeroed counters and the slot record, in one copy; the
    // slot is published only once they are on the device.
    char *h = static_cast<char *>(hstage_[slot]);
    std::memcpy(h, st.data(), st.size() * sizeof(EngStage));
    std::memset(h + stage_bytes_, 0, sizeof(EngCounters) * st.size());
    EngSlot rec{(int)st.size(), 0, g, 0};
    std::memcpy(h + stage_bytes_ + sizeof(EngCounters) * max_stages_, &rec, sizeof(rec));
    const size_t off = (size_t)slot * max_stages_;
    CHASE_HIP(hipMemcpyAsync(dstages_ + off, h, st.size() * sizeof(EngStage),
                             hipMemcpyHostToDevice, cs_));
    CHASE_HIP(hipMemcpyAsync(dcnt_ + off, h + stage_bytes_, st.size() * sizeof(EngCounters),
                             hipMemcpyHostToDevice, cs_));
    CHASE_HIP(hipMemcpyAsync(dslots_ + slot, h + stage_bytes_ + sizeof(EngCounters) * max_stages_,
                             sizeof(EngSlot), hipMemcpyHostToDevice, cs_));
    CHASE_HIP(hipStreamSynchronize(cs_));
    __atomic_store_n(&ctl_->gen[slot], g, __ATOMIC_SEQ_CST);
    __atomic_fetch_or(&ctl_->active, 1ull << slot, __ATOMIC_SEQ_CST);
    if (kernel_exited_locked()) launch_locked();
    items_ += 0;
    for (const EngStage &S : st) items_ += S.tiles + S.reduces;
    ++jobs_;
    return slot;
}

void FilterEngine::wait(int slot) {
    // The job is done when the kernel says so.  The kernel may also have
    // left on its own (its idle backstop) while the job was being
    // published: then it is launched again.
    const auto t0 = std::chrono::steady_clock::now();
    auto t_last = t0;
    int spins = 0, relaunches = 0;
    while (__atomic_load_n(&ctl_->done[slot], __ATOMIC_ACQUIRE) == 0) {
        if (++spins < 64) {
            std::this_thread::yield();
            continue;
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        const auto now = std::chrono::steady_clock::now();
        if (now - t_last > std::chrono::milliseconds(100)) {
            t_last = now;
            std::lock_guard<std::mutex> lk(mu_);
            if (__atomic_load_n(&ctl_->done[slot], __ATOMIC_ACQUIRE) == 0) {
                if (kernel_exited_locked()) {
                    // A job the kernel could not finish in two lifetimes is
                    // not coming: give up rather than wait for ever.
                    if (++relaunches > 2) {
                        busy_[slot] = false;
                        --active_;
                        __atomic_fetch_and(&ctl_->active, ~(1ull << slot), __ATOMIC_SEQ_CST);
                        cv_.notify_all();
                        throw Error(3, "filter engine: a job did not complete");
                    }
                    launch_locked();
                }
                if (now - t0 > std::chrono::seconds(900)) {
                    // Past any filter call's duration: stop the kernel (its
                    // workgroups leave when idle or at their spin limits).
                    busy_[slot] = false;
                    --active_;
                    __atomic_fetch_and(&ctl_->active, ~(1ull << slot), __ATOMIC_SEQ_CST);
                    stop_kernel_locked();
                    cv_.notify_all();
                    throw Error(3, "filter engine: a job did not complete in 900 s");
                }
            }
        }
    }
    std::lock_guard<std::mutex> lk(mu_);
    __atomic_fetch_and(&ctl_->active, ~(1ull << slot), __ATOMIC_SEQ_CST);
    busy_[slot] = false;
    --active_;
    const int err = __atomic_load_n(&ctl_->err, __ATOMIC_ACQUIRE);
    // With no job left the kernel is stopped (it would only poll).
    if (active_ == 0) stop_kernel_locked();
    cv_.notify_all();
    if (err) throw Error(3, "filter engine: a job could not be run");
}

void FilterEngine::stats(int64_t *jobs, int64_t *items, int64_t *launches) {
    std::lock_guard<std::mutex> lk(mu_);
    if (jobs) *jobs = jobs_;
    if (items) *items = items_;
    if (launches) *launches = launches_;
}

}  // namespace chase
