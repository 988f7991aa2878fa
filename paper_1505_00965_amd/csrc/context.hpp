// Library context: device, stream, device buffers and the last error.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/mlmc.h"
#include "level.hpp"

struct mlmc_ctx {
    int device = 0;
    int num_cu = 256;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    std::string err;
    int launch_block = 0, launch_ppt = 0;   // 0: tuned/default
    int persist_block = 0, persist_ppt = 0, persist_bpc = 0;
    void* persist = nullptr;                // persistent-form buffers (persistent.hip)
    // Level accumulators: kAccSlots records (payoff x level) + host mirror.
    mlmc::LevelAcc* d_acc = nullptr;
    mlmc::LevelAcc* h_acc = nullptr;
    // Driver state on the device and its pinned host mirror (driver.hip).
    void* d_drv = nullptr;
    void* h_drv = nullptr;        // pinned host mirror of the driver state
    void* h_drv_dev = nullptr;    // the same memory as the device sees it
    // spread groups of the per-level launches, one per level (driver.hip)
    mlmc::LevelAcc* d_drv_spread = nullptr;
    // the groups are known to hold zeros: the last run ended normally (its
    // updates folded and cleared every group it used)
    bool drv_clean = false;
    // the driver state and the plan table hold a fresh start for the next
    // device-planned run of the same descriptor (the last call was one, and
    // the update queued past its end prepared it)
    bool drv_pilot_ready = false;
    double* d_tmp = nullptr;                // small fp64 scratch (optimal_n)
    double* h_tmp = nullptr;
    // kernel timing (mlmc_set_timing)
    struct Timed {
        hipEvent_t start, stop;
        int slot;
        double fine_steps, coarse_steps;
    };
    uint32_t timing = 0;                    // bit s: time launches of slot s
    uint32_t timing_stride = 1;             // time one launch in this many of a slot
    bool timing_paused = false;             // stamp nothing for now (mask and stats kept)
    uint64_t timing_seen[MLMC_STAT_SLOTS] = {};   // launches of each slot since the mask was set
    std::vector<hipEvent_t> event_pool;
    std::vector<Timed> pending;
    mlmc_kernel_stat stats[MLMC_STAT_SLOTS] = {};
    // tuned launch shapes (autotune.cpp), keyed by kernel and problem class
    std::map<std::string, std::vector<int>> tuned;
};

namespace mlmc {

// Level records: 16 spread groups (a call's level, or every level of a
// randomised single-term estimate); also the training records and the host
// copy of a persistent batch.
constexpr int kAccSlots = 16 * mlmc::kSpread;

// Record an error message and return the status.
mlmc_status fail(mlmc_ctx* ctx, mlmc_status st, const std::string& msg);
mlmc_status hip_fail(mlmc_ctx* ctx, hipError_t e, const char* what);

#define MLMC_HIP(ctx, expr)                                              \
    do {                                                                 \
        hipError_t e__ = (expr);                                         \
        if (e__ != hipSuccess) return ::mlmc::hip_fail((ctx), e__, #expr); \
    } while (0)

// Argument validation shared by the level entry points.
// Path steps per sample of level l (n_f + n_c; 2 n_f + n_c with the twin).
double level_cost(const mlmc_model& m, int l, int M);
mlmc_status check_level_args(mlmc_ctx* ctx, const mlmc_model* m, const mlmc_payoff* p, int l, int M,
                             int precision);
// The same checks without a context: the reason (a static string) or null.
const char* level_args_error(const mlmc_model* m, const mlmc_payoff* p, int l, int M, int precision);
// Launch shape for N samples at level l (honours mlmc_set_launch); paths
// are split across lanes by the count of the whole call, n_call >= N (a call
// may be cut into several launches at the counter's high word).
LaunchShape choose_shape(const mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l,
                         int M, int precision, uint64_t N, uint64_t n_call = 0);
// The rule behind choose_shape, from its inputs alone: a fixed shape
// (fixed_block != 0), else a tuned one (tuned_block != 0), else 256 threads
// and 2 samples per lane; one sample per lane when fewer than 256 lanes per
// compute unit would be busy; one- and two-step levels at most 2 blocks per
// lane; GBM paths split across lanes when too few fill the device.  The
// returned shape has no residency cap (num_cu = 0).
LaunchShape default_shape(const mlmc_model& m, const mlmc_payoff& p, int l, int M, int precision,
                          uint64_t N, uint64_t n_call, int num_cu, int fixed_block, int fixed_ppt,
                          int tuned_block, int tuned_ppt);
// One plain-sampler launch over a range whose generator units share their
// counter word 2 (no control variate): arguments as for enqueue_level.
hipError_t launch_plain_segment(const mlmc_model& m, const mlmc_payoff& p, int l, int M, uint64_t N,
                                uint64_t seed, uint64_t offset, int precision, uint32_t stream,
                                int coupled, LevelAcc* acc, double* d_pf, double* d_pc, bool spread,
                                const LaunchShape& shape, hipStream_t st, hipEvent_t t0 = nullptr,
                                hipEvent_t t1 = nullptr);
// Enqueue one level into record `acc`, or with `spread` into the spread
// group of kSpread records at `acc` (no zeroing, no sync).
mlmc_status enqueue_level(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l, int M,
                          uint64_t N, uint64_t seed, uint64_t offset, int precision, uint32_t stream,
                          int coupled, LevelAcc* acc, double* d_pf, double* d_pc,
                          const mlmc_cv* cv, bool spread = false);
// Zero `n` records with a fill kernel (safe inside graph capture).
hipError_t zero_records(LevelAcc* acc, int n, hipStream_t st);

// Bracket a launch with timing events when timing is on (no-op otherwise).
// timed_begin returns an index for timed_end, or -1.
int timed_begin(mlmc_ctx* ctx, int slot, double fine_steps, double coarse_steps);
void timed_end(mlmc_ctx* ctx, int idx);
// Event pair for a kernel launched with start/stop events (nullptr, nullptr
// when timing is off); harvested like timed_begin's.
void timed_kernel(mlmc_ctx* ctx, int slot, double fine_steps, double coarse_steps,
                  hipEvent_t* start, hipEvent_t* stop);
// After the stream has been synchronised: fold finished events into stats.
void harvest_timing(mlmc_ctx* ctx);
// Fold in the stamped launches that have finished, without waiting for the
// stream (the rest stay pending until a later harvest).
void harvest_ready(mlmc_ctx* ctx);

// Release the driver state and the persistent batch buffers (idempotent).
void free_driver(mlmc_ctx* ctx);
void free_persistent(mlmc_ctx* ctx);

// Tuned shape of the level sampler for this problem, if the tuner ran.
bool tuned_shape(const mlmc_ctx* ctx, const mlmc_model& m, int payoff, int precision, int M, int l,
                 int* block, int* ppt);
int level_class(int l, int M);

// Control variate (cv.hip).
// tab: the tabulated network (estimation launches of a network switched to
// it); training launches always evaluate the network itself.
hipError_t cv_ensure_phi0(const mlmc_cv* cv, const mlmc_model& m, hipStream_t st, bool tab);
bool cv_tabulated(const mlmc_cv* cv);
hipError_t cv_launch_level(const mlmc_cv* cv, const mlmc_model& m, const mlmc_payoff& p, int M,
                           const LevelArgs<float>& a, int grid, hipStream_t st, bool tab, int ppt = 1);
const float* cv_phi0_ptr(const mlmc_cv* cv, bool tab);
int cv_in_dim(const mlmc_cv* cv);

hipError_t launch_philox_words(uint64_t seed, int level, uint64_t s0, uint32_t stream,
                               uint32_t nblocks, uint64_t npaths, uint32_t* out, hipStream_t st);
hipError_t launch_normals(uint64_t seed, int level, uint64_t s0, uint32_t stream, int dim,
                          int nsteps, uint64_t npaths, int precision, double* out, hipStream_t st);

}  // namespace mlmc
