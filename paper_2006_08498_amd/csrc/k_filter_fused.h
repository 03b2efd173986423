// Persistent filter engine (k_filter_fused.hip): the FP64 filter calls of
// several eigenproblems run by one long-lived kernel as they arrive.
#pragma once

#include "common.h"

#include <condition_variable>
#include <mutex>
#include <vector>

namespace chase {

constexpr int kEngineSlots = 64;        // jobs in flight at once
constexpr int kEngineMaxStages = 512;   // stages (steps x column pieces) per job

struct EngStage;
struct EngCounters;
struct EngCtl;
struct EngSlot;

// A job is the list of FilterCall steps of one filter call, in the order
// filter_steps gives them; its result is bitwise the one filter_gemm step
// by step gives.  submit() returns once the job is handed to the device
// (its input data must be complete and stay valid until wait() returns);
// wait() blocks until the job's results are in memory, visible to kernels
// launched afterwards.  Thread-safe; one engine per device.  The kernel runs
// while jobs are in flight and is stopped when none is left.
class FilterEngine {
  public:
    FilterEngine();
    ~FilterEngine();
    FilterEngine(const FilterEngine &) = delete;
    FilterEngine &operator=(const FilterEngine &) = delete;

    int submit(const std::vector<FilterCall> &steps);
    void wait(int slot);
    void stats(int64_t *jobs, int64_t *items, int64_t *launches);

  private:
    void launch_locked();
    bool kernel_exited_locked();
    void stop_kernel_locked();

    std::mutex mu_;
    std::condition_variable cv_;
    int device_ = -1;
    hipStream_t ks_ = nullptr, cs_ = nullptr;   // kernel, descriptor copies
    hipEvent_t kdone_ = nullptr;
    bool running_ = false;
    EngCtl *ctl_ = nullptr;
    EngSlot *dslots_ = nullptr;
    EngStage *dstages_ = nullptr;
    EngCounters *dcnt_ = nullptr;
    void *hstage_[kEngineSlots] = {};
    size_t stage_bytes_ = 0;
    int max_stages_ = 0;
    int grid_ = 0;
    bool busy_[kEngineSlots] = {};
    int gen_[kEngineSlots] = {};
    int active_ = 0;
    int64_t jobs_ = 0, items_ = 0, launches_ = 0;
};

int fused_tile_width();

}  // namespace chase
