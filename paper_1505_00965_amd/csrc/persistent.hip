// Persistent all-levels sampler: every level (and payoff) of one MLMC
// iteration in a single launch, captured once in a HIP graph.
//
// Levels are independent (Sec. 5, after eq. (eq:Yldef)), so one iteration's
// work is a set of (payoff, level, sample range) items.  Their costs differ by
// orders of magnitude: level l costs M^l + M^(l-1) steps per sample (the
// paper's cost measure, Sec. 3) and N_l falls with l.  A plan kernel cuts the
// outstanding samples into items of roughly equal cost, deepest levels first
// (longest-processing-time order), and a resident grid of blocks takes items
// (block b item b first, then from an atomic counter) until none are left, so
// cheap levels fill in around the long deep-level items.  GBM levels with too few paths to fill the
// device run each path on several lanes (process_split), with the per-level
// launch's rule on the level's count.  Every parameter the launches read lives in
// device memory and is rewritten between launches (by the driver kernel or
// by host copies), so the graph is captured once and replayed.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "context.hpp"
#include "driver.hpp"
#include "sampler_impl.hpp"
#include "trace.hpp"

namespace mlmc {

constexpr int kMaxSlots = 4;          // payoffs per batch
constexpr int kItemsPerBlock = 4;     // target items per resident block
constexpr unsigned kItemsPerPair = 1024;
constexpr unsigned kMaxItems = kMaxSlots * kMaxLevels * kItemsPerPair;

struct WorkItem {
    uint64_t first;     // first sample index of the range
    uint32_t n;         // number of samples
    uint16_t level;
    uint8_t slot;       // payoff slot
    uint8_t pad;
};

// Device-resident batch description (rewritten before each launch).
struct BatchDesc {
    int nslots, L, M, pad;
    int payoff_kind[kMaxSlots];
    StepParams<float> params[kMaxSlots][kMaxLevels];
    uint64_t seed;
    // outstanding samples and their first index, per (slot, level); for the
    // driver these alias DriverState::dN / n (slot 0 only)
    const double* dN;
    const double* offset;
    LevelAcc* acc;                    // spread groups [slot][level][kSpread]
    WorkItem* items;
    unsigned* head;                   // dispenser of the items past the first gridDim.x
    unsigned* count;                  // number of items
    unsigned resident_blocks;         // grid size of the sampler
    unsigned chunk;                   // blockDim * PPT of the sampler
    unsigned block;                   // blockDim of the sampler
    unsigned* split;                  // lanes per path per (slot, level), set by the plan
    int split_ok;                     // the model's paths are linear in their start (GBM)
    int num_cu;
};

// Plan: the first wave sizes the (slot, level) pairs, one lane each, in
// processing order (deepest level first, then slot), so the independent
// global reads and the 64-bit divisions run side by side; a wave scan gives
// each pair its first item, and the block then writes the items in parallel.
// Every thread of the block must call it.
__device__ __forceinline__ void plan_body(const BatchDesc* d)
{
    constexpr int kPairs = kMaxSlots * kMaxLevels;
    static_assert(kPairs == 64, "one lane of the first wave per (slot, level) pair");
    __shared__ uint64_t s_first[kPairs], s_left[kPairs], s_per[kPairs];
    __shared__ unsigned s_start[kPairs + 1];
    __shared__ int s_slot[kPairs], s_level[kPairs];
    __shared__ int s_npairs;
    if (threadIdx.x < 64) {
        const int L = d->L, M = d->M, nslots = d->nslots;
        const int p = (int)threadIdx.x;
        const bool valid = p < (L + 1) * nslots;
        const int l = valid ? L - p / nslots : 0, s = valid ? p % nslots : 0;
        double nf = 1.0;
        for (int i = 0; i < l; ++i) nf *= M;   // M^l, exact
        const double per = nf + (l ? nf / M : 0.0);
        const double dn = valid ? d->dN[s * kMaxLevels + l] : 0.0;
        // samples x steps over the batch (lane 0's sum: the rotations leave
        // other lanes with other association orders)
        const double total = __shfl(wave_sum(valid ? dn * per : 0.0), 0);
        const double target = total / ((double)d->resident_blocks * kItemsPerBlock);
        const uint64_t left = (uint64_t)dn;
        unsigned items = 0;
        uint64_t per_item = 0;
        if (valid) {
            // lanes per path: the per-level launch's rule on the same count
            const uint32_t G = split_lanes((int)nf, left, d->num_cu,
                                           d->split_ok && d->payoff_kind[s] != kDigitalCond);
            d->split[s * kMaxLevels + l] = G;
            if (left) {
                uint64_t paths = (uint64_t)(target / per);
                if (G > 1) {
                    // split paths: whole block passes of block / G paths
                    const uint64_t pass = d->block / G;
                    paths = paths < pass ? pass : (paths / pass) * pass;
                } else if (paths >= d->chunk) {
                    paths = (paths / d->chunk) * d->chunk;   // whole chunks where possible
                } else if (paths < d->block) {
                    paths = d->block;                        // one sample per lane at least
                }
                if (paths > (1ull << 31)) paths = 1ull << 31;   // item counts fit 32 bits
                // at most kItemsPerPair items per pair: the table never fills
                const uint64_t min_items = (left + kItemsPerPair - 1) / kItemsPerPair;
                per_item = paths > min_items ? paths : min_items;
                items = (unsigned)((left + per_item - 1) / per_item);
            }
        }
        // exclusive scan of the item counts over the lanes (pair order)
        unsigned incl = items;
#pragma unroll
        for (int k = 1; k < 64; k <<= 1) {
            const unsigned v = __shfl_up(incl, k);
            if (p >= k) incl += v;
        }
        // pairs with samples, packed in order
        const uint64_t active = __ballot(items > 0);
        const int rank = __popcll(active & ((1ull << p) - 1ull));
        if (items) {
            s_first[rank] = (uint64_t)d->offset[s * kMaxLevels + l];
            s_left[rank] = left;
            s_per[rank] = per_item;
            s_slot[rank] = s;
            s_level[rank] = l;
            s_start[rank] = incl - items;
        }
        if (p == 63) {
            const int np = __popcll(active);
            s_start[np] = incl;
            s_npairs = np;
            *d->count = incl;
            *d->head = 0;
        }
    }
    __syncthreads();
    const int np = s_npairs;
    const unsigned count = s_start[np];
    for (unsigned k = threadIdx.x; k < count; k += blockDim.x) {
        int q = 0;
        while (q + 1 < np && s_start[q + 1] <= k) ++q;
        const uint64_t i = k - s_start[q];
        const uint64_t done = i * s_per[q];
        const uint64_t n = s_left[q] - done < s_per[q] ? s_left[q] - done : s_per[q];
        WorkItem w;
        w.first = s_first[q] + done;
        w.n = (uint32_t)n;
        w.level = (uint16_t)s_level[q];
        w.slot = (uint8_t)s_slot[q];
        w.pad = 0;
        d->items[k] = w;
    }
}

__global__ __launch_bounds__(256) void plan_kernel(const BatchDesc* d) { plan_body(d); }

// Fold each spread group (kSpread records) into one record, group g by
// block g, in record order; clears the groups for the next replay.
__global__ __launch_bounds__(64) void fold_groups_kernel(LevelAcc* groups, LevelAcc* out)
{
    static_assert(kSpread == 64, "one lane per record of a group");
    LevelAcc& r = groups[blockIdx.x * kSpread + threadIdx.x];
    double v[kNumSums];
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] = wave_sum(r.sum[k]);
    const double c = wave_sum((double)r.n_nonfinite);
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) r.sum[k] = 0.0;
    r.n_nonfinite = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) out[blockIdx.x].sum[k] = v[k];
        out[blockIdx.x].n_nonfinite = (unsigned long long)c;
        out[blockIdx.x].pad = 0;
    }
}

// The samples [a.offset, a.offset + a.N) of one item part (a.c2, a.c2b set).
template <int MODEL, int PAYOFF, int M, int PPT>
__device__ __forceinline__ void run_range(const LevelArgs<float>& a, double (&sums)[kNumSums],
                                          unsigned& nonfinite)
{
    if constexpr (MODEL != kHeston && PAYOFF != kDigitalCond) {
        if (a.split > 1) {
            const uint64_t pass = blockDim.x / a.split;
            for (uint64_t base = 0; base < a.N; base += pass)
                process_split<MODEL, PAYOFF, M>(a, base, sums, nonfinite);
            return;
        }
    }
    if (a.nf < 4) {
        // one or two steps: samples share generator blocks
        constexpr int D = one_factor(MODEL) ? 1 : 2;
        const int q = 4 / (a.nf * D);
        const uint64_t nblk = short_blocks(a.offset, a.N, q);
        const uint64_t chunk = (uint64_t)blockDim.x * PPT;
        const FullChunks f = full_chunks(a.offset, a.N, q, chunk);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(f.lo), hi = __builtin_amdgcn_readfirstlane(f.hi);
        // one counter segment: chunk indices fit 32 bits (a scalar loop test)
        const uint32_t nch = __builtin_amdgcn_readfirstlane((uint32_t)((nblk + chunk - 1) / chunk));
        for (uint32_t c = 0; c < nch; ++c) {
            const uint64_t base = (uint64_t)c * chunk;
            const bool full = c >= lo && c < hi;
            if (a.nf == 1) process_short<MODEL, PAYOFF, float, 1, M, PPT, false>(a, base, full, sums, nonfinite);
            else process_short<MODEL, PAYOFF, float, 2, M, PPT, false>(a, base, full, sums, nonfinite);
        }
    } else if (a.N <= blockDim.x) {
        // fewer samples than lanes: one per lane
        process_chunk<MODEL, PAYOFF, float, M, 1, false>(a, 0, sums, nonfinite);
    } else {
        const uint64_t chunk = (uint64_t)blockDim.x * PPT;
        for (uint64_t base = 0; base < a.N; base += chunk)
            process_chunk<MODEL, PAYOFF, float, M, PPT, false>(a, base, sums, nonfinite);
    }
}

template <int MODEL, int PAYOFF, int M, int PPT>
__device__ __forceinline__ void run_item(const BatchDesc* d, const WorkItem& w, double (&sums)[kNumSums],
                         unsigned& nonfinite)
{
    LevelArgs<float> a;
    a.P = d->params[w.slot][w.level];
    a.seed = d->seed;
    a.l = w.level;
    int nf = 1;
    for (int i = 0; i < a.l; ++i) nf *= M;
    a.nf = nf;
    a.ngroups = (uint32_t)((nf + 3) / 4);
    a.stream = kStreamNormal;
    a.acc = nullptr;
    a.pf_out = a.pc_out = nullptr;
    a.coupled = 1;
    a.phi0 = nullptr;
    a.split = d->split[w.slot * kMaxLevels + w.level];
    constexpr int D = one_factor(MODEL) ? 1 : 2;
    // one pass per part of the item whose generator units share counter word 2
    const uint64_t q = samples_per_unit(nf, D), end = w.first + w.n;
    for (uint64_t first = w.first; first < end;) {
        const uint64_t stop = counter_segment_end(first, end, q);
        a.offset = first;
        a.N = stop - first;
        set_counter_words(a, D);
        run_range<MODEL, PAYOFF, M, PPT>(a, sums, nonfinite);
        first = stop;
    }
}

// Block b takes item b first; later items come from the dispenser until
// none are left, so a launch with no more items than blocks (an empty one
// included) makes no atomics on it.  Each item ends with a block reduction
// into its (payoff, level) spread group.
template <int MODEL, int M, int PPT>
__device__ __forceinline__ void sample_items(const BatchDesc* d)
{
    __shared__ unsigned s_item;
    const unsigned count = *d->count;
    for (unsigned it = blockIdx.x; it < count;) {   // block-uniform
        const WorkItem w = d->items[it];
        double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
        unsigned nonfinite = 0;
        switch (d->payoff_kind[w.slot]) {
        case kCall: run_item<MODEL, kCall, M, PPT>(d, w, sums, nonfinite); break;
        case kAsian: run_item<MODEL, kAsian, M, PPT>(d, w, sums, nonfinite); break;
        case kLookback: run_item<MODEL, kLookback, M, PPT>(d, w, sums, nonfinite); break;
        case kDigitalCond: run_item<MODEL, kDigitalCond, M, PPT>(d, w, sums, nonfinite); break;
        default: run_item<MODEL, kDigital, M, PPT>(d, w, sums, nonfinite); break;
        }
        if (w.level == 0) copy_y_sums(sums);
        block_reduce_add(sums, nonfinite, &d->acc[(w.slot * kMaxLevels + w.level) * kSpread +
                                                  (blockIdx.x & (kSpread - 1))]);
        if (count <= gridDim.x) break;
        if (threadIdx.x == 0) s_item = gridDim.x + atomicAdd(d->head, 1u);
        __syncthreads();
        it = s_item;
        __syncthreads();
    }
}

template <int MODEL, int M, int PPT>
__global__ __launch_bounds__(1024) void persistent_kernel(const BatchDesc* d)
{
    sample_items<MODEL, M, PPT>(d);
}

using PersistentFn = void (*)(const BatchDesc*);

template <int MODEL, int M>
static PersistentFn pick_ppt(int ppt)
{
    switch (ppt) {
    case 1: return persistent_kernel<MODEL, M, 1>;
    case 2: return persistent_kernel<MODEL, M, 2>;
    default: return persistent_kernel<MODEL, M, 4>;
    }
}

// variant: sampler_variant() of the model (GBM Euler, GBM Milstein, Heston)
static PersistentFn pick_persistent(int variant, int M, int ppt)
{
    if (variant == kGBM) return M == 2 ? pick_ppt<kGBM, 2>(ppt) : pick_ppt<kGBM, 4>(ppt);
    if (variant == kGBMMil) return M == 2 ? pick_ppt<kGBMMil, 2>(ppt) : pick_ppt<kGBMMil, 4>(ppt);
    return M == 2 ? pick_ppt<kHeston, 2>(ppt) : pick_ppt<kHeston, 4>(ppt);
}


// Device buffers of the persistent form, owned by the context.
struct PersistentBufs {
    BatchDesc* d_desc = nullptr;
    BatchDesc* h_desc = nullptr;
    WorkItem* d_items = nullptr;
    unsigned* d_counters = nullptr;   // head, count
    LevelAcc* d_acc = nullptr;        // batch spread groups [kMaxSlots][kMaxLevels][kSpread]
    LevelAcc* d_rec = nullptr;        // their folds [kMaxSlots][kMaxLevels]
    unsigned* d_split = nullptr;      // lanes per path [kMaxSlots][kMaxLevels]
    double* d_req = nullptr;          // dN[kMaxSlots][kMaxLevels], offset[...]
    double* h_req = nullptr;
    hipGraphExec_t graph = nullptr;   // cached batch graph
    int graph_key[5] = {-1, -1, -1, -1, -1};
    hipGraphExec_t run_graph = nullptr;   // cached driver-iteration graph
    int run_key[5] = {-1, -1, -1, -1, -1};
    BatchDesc last_desc;              // the bytes of the last descriptor upload
    bool last_ok = false;
};

static PersistentBufs* bufs_of(mlmc_ctx* ctx);

struct PersistentShape {
    int block, ppt, blocks_per_cu;
};

static PersistentShape persistent_shape(const mlmc_ctx* ctx)
{
    PersistentShape s;
    s.block = ctx->persist_block ? ctx->persist_block : 256;
    s.ppt = ctx->persist_ppt ? ctx->persist_ppt : 1;
    s.blocks_per_cu = ctx->persist_bpc ? ctx->persist_bpc : 4;
    return s;
}

static mlmc_status ensure_bufs(mlmc_ctx* ctx)
{
    if (ctx->persist) return MLMC_OK;
    auto* b = new (std::nothrow) PersistentBufs();
    if (!b) return fail(ctx, MLMC_ENOMEM, "host allocation failed");
    ctx->persist = b;
    hipError_t e = hipMalloc(&b->d_desc, sizeof(BatchDesc));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_desc, sizeof(BatchDesc));
    if (e == hipSuccess) e = hipMalloc(&b->d_items, sizeof(WorkItem) * kMaxItems);
    if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(unsigned) * 4);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_acc, sizeof(LevelAcc) * kMaxSlots * kMaxLevels * kSpread);
    if (e == hipSuccess) e = hipMalloc(&b->d_rec, sizeof(LevelAcc) * kMaxSlots * kMaxLevels);
    if (e == hipSuccess) e = hipMalloc(&b->d_split, sizeof(unsigned) * kMaxSlots * kMaxLevels);
    if (e == hipSuccess) e = hipMalloc(&b->d_req, sizeof(double) * 2 * kMaxSlots * kMaxLevels);
    if (e == hipSuccess)
        e = hipHostMalloc(&b->h_req, sizeof(double) * 2 * kMaxSlots * kMaxLevels);
    if (e != hipSuccess) {
        // An incomplete set is released so that the next call starts over.
        free_persistent(ctx);
        return hip_fail(ctx, e, "persistent batch allocation");
    }
    return MLMC_OK;
}

static PersistentBufs* bufs_of(mlmc_ctx* ctx) { return (PersistentBufs*)ctx->persist; }

void free_persistent(mlmc_ctx* ctx)
{
    auto* b = bufs_of(ctx);
    if (!b) return;
    if (b->graph) hipGraphExecDestroy(b->graph);
    if (b->run_graph) hipGraphExecDestroy(b->run_graph);
    if (b->d_desc) hipFree(b->d_desc);
    if (b->h_desc) hipHostFree(b->h_desc);
    if (b->d_items) hipFree(b->d_items);
    if (b->d_counters) hipFree(b->d_counters);
    if (b->d_acc) hipFree(b->d_acc);
    if (b->d_rec) hipFree(b->d_rec);
    if (b->d_split) hipFree(b->d_split);
    if (b->d_req) hipFree(b->d_req);
    if (b->h_req) hipHostFree(b->h_req);
    delete b;
    ctx->persist = nullptr;
}

// Fill the host copy of the descriptor (parameters for every slot and level).
static void fill_desc(mlmc_ctx* ctx, BatchDesc* h, const mlmc_model& m, const mlmc_payoff* p,
                      int np, int L, int M, uint64_t seed, const double* dN, const double* off,
                      LevelAcc* acc)
{
    auto* b = bufs_of(ctx);
    const PersistentShape s = persistent_shape(ctx);
    std::memset(h, 0, sizeof(*h));
    h->nslots = np;
    h->L = L;
    h->M = M;
    for (int k = 0; k < np; ++k) {
        h->payoff_kind[k] = p[k].kind;
        for (int l = 0; l <= L; ++l) h->params[k][l] = make_step_params<float>(m, p[k], l, M);
    }
    h->seed = seed;
    h->dN = dN;
    h->offset = off;
    h->acc = acc;
    h->items = b->d_items;
    h->head = b->d_counters;
    h->count = b->d_counters + 1;
    h->resident_blocks = (unsigned)(ctx->num_cu * s.blocks_per_cu);
    h->chunk = (unsigned)(s.block * s.ppt);
    h->split = b->d_split;
    h->split_ok = m.kind == MLMC_GBM && !m.antithetic;
    h->num_cu = ctx->num_cu;
    h->block = (unsigned)s.block;
}

// Copy the host descriptor to the device unless the last upload from this
// context carried the same bytes (repeated runs of one problem skip it).
static mlmc_status upload_desc(mlmc_ctx* ctx, PersistentBufs* b)
{
    if (b->last_ok && std::memcmp(&b->last_desc, b->h_desc, sizeof(BatchDesc)) == 0)
        return MLMC_OK;
    b->last_ok = false;
    MLMC_HIP(ctx, hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice,
                                 ctx->stream));
    std::memcpy(&b->last_desc, b->h_desc, sizeof(BatchDesc));
    b->last_ok = true;
    return MLMC_OK;
}

// Capture [prologue?] -> plan -> persistent -> [epilogue] into a graph.
static mlmc_status capture(mlmc_ctx* ctx, int model, int M, bool zero_batch,
                           DriverState* driver, hipGraphExec_t* out)
{
    auto* b = bufs_of(ctx);
    const PersistentShape s = persistent_shape(ctx);
    hipStream_t cs;
    MLMC_HIP(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && zero_batch)
        e = zero_records(b->d_acc, kMaxSlots * kMaxLevels * kSpread, cs);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(256), 0, cs, (const BatchDesc*)b->d_desc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pick_persistent(model, M, s.ppt), dim3(ctx->num_cu * s.blocks_per_cu),
                           dim3(s.block), 0, cs, (const BatchDesc*)b->d_desc);
        e = hipGetLastError();
    }
    if (e == hipSuccess && zero_batch) {
        hipLaunchKernelGGL(fold_groups_kernel, dim3(kMaxSlots * kMaxLevels), dim3(kSpread), 0, cs,
                           b->d_acc, b->d_rec);
        e = hipGetLastError();
    }
    if (e == hipSuccess && driver)
        e = launch_driver_update(driver, (DriverState*)ctx->h_drv_dev, ctx->d_drv_spread, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent graph capture");
    return MLMC_OK;
}

// mlmc_run with persistent = 1: one graph launch per driver iteration.
mlmc_status run_persistent(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p,
                           const mlmc_run_opts& o, DriverState* d_st, DriverState* h_st)
{
    if (o.precision != 32) return fail(ctx, MLMC_EINVAL, "the persistent form runs fp32 paths");
    if (o.cv) return fail(ctx, MLMC_EINVAL, "the persistent form runs plain MLMC");
    mlmc_status st = ensure_bufs(ctx);
    if (st) return st;
    auto* b = bufs_of(ctx);
    fill_desc(ctx, b->h_desc, m, &p, 1, o.L_max, o.M, o.seed, d_st->dN, d_st->n,
              ctx->d_drv_spread);
    st = upload_desc(ctx, b);
    if (st) return st;
    // the graph reads the descriptor, the driver state and its mirror at
    // replay, all fixed per context: one capture serves every run
    const PersistentShape s = persistent_shape(ctx);
    const int key[5] = {sampler_variant(m), o.M, s.block, s.ppt, s.blocks_per_cu};
    if (!b->run_graph || std::memcmp(key, b->run_key, sizeof(key)) != 0) {
        // an earlier run may return with its last (empty) launch queued
        MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (b->run_graph) hipGraphExecDestroy(b->run_graph);
        b->run_graph = nullptr;
        st = capture(ctx, sampler_variant(m), o.M, false, d_st, &b->run_graph);
        if (st) return st;
        std::memcpy(b->run_key, key, sizeof(key));
    }
    hipGraphExec_t g = b->run_graph;
    // Iteration k + 1 is enqueued before the host waits for iteration k's
    // update: its plan reads the batch that update set from the device
    // state, so the GPU runs the iterations back to back while the host reads
    // the mirror.  The one launch past the last update finds the driver done
    // and does nothing (no outstanding batch; the update leaves the state).
    int first_tix = -1;
    for (int it = 0;; ++it) {
        if (it > h_st->max_iterations + 1)
            return fail(ctx, MLMC_EDEVICE, "driver state did not reach the host");
        const TraceRange iter_range("mlmc_run driver iteration (graph)");
        for (int k = it ? 1 : 0; k < 2; ++k) {
            const int tix = timed_begin(ctx, 16, 0.0, 0.0);
            if (first_tix < 0) first_tix = tix;
            const hipError_t e = hipGraphLaunch(g, ctx->stream);
            timed_end(ctx, tix);
            if (e != hipSuccess) return hip_fail(ctx, e, "persistent iteration");
        }
        // the update kernel inside the graph also writes the host mirror h_st
        const hipError_t e = wait_update(ctx->stream, h_st, (unsigned long long)it + 1);
        if (e != hipSuccess) return hip_fail(ctx, e, "persistent iteration");
        // the flag comes in the word that publishes the update, so a mirror
        // seen done is complete; later updates leave it as it is
        if (mirror_done(h_st)) break;
    }
    // the launch past the last update may still run: the result is read from
    // the mirror, and the stream is waited for only to read timing events
    if (ctx->pending.empty()) return MLMC_OK;
    const hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent iteration");
    if (first_tix >= 0) {
        // the launches' path steps are known only as a whole: every sampled
        // batch is absorbed into n_l, so they are charged to the first entry
        double fine = 0.0, coarse = 0.0;
        for (int l = 0; l <= h_st->L; ++l) {
            const double nf = std::pow((double)o.M, (double)l);
            fine += h_st->n[l] * nf;
            coarse += l ? h_st->n[l] * nf / o.M : 0.0;
        }
        ctx->pending[first_tix].fine_steps = fine;
        ctx->pending[first_tix].coarse_steps = coarse;
    }
    harvest_timing(ctx);
    return MLMC_OK;
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

mlmc_status mlmc_set_persistent_launch(mlmc_ctx* ctx, int block, int ppt, int blocks_per_cu)
{
    if (!ctx) return MLMC_EINVAL;
    if (block == 0) {
        ctx->persist_block = ctx->persist_ppt = ctx->persist_bpc = 0;
    } else {
        if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
            return fail(ctx, MLMC_EINVAL, "block must be 64, 128, 256, 512 or 1024");
        if (ppt != 1 && ppt != 2 && ppt != 4) return fail(ctx, MLMC_EINVAL, "ppt must be 1, 2 or 4");
        if (blocks_per_cu < 1 || blocks_per_cu * block > 4096)
            return fail(ctx, MLMC_EINVAL, "blocks_per_cu * block must be in 1..4096 threads");
        ctx->persist_block = block;
        ctx->persist_ppt = ppt;
        ctx->persist_bpc = blocks_per_cu;
    }
    if (auto* b = bufs_of(ctx)) {
        // a run may have returned with its last (empty) launch queued
        MLMC_HIP(ctx, hipSetDevice(ctx->device));
        MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (b->graph) hipGraphExecDestroy(b->graph);
        if (b->run_graph) hipGraphExecDestroy(b->run_graph);
        b->graph = b->run_graph = nullptr;
        b->graph_key[0] = b->run_key[0] = -1;
    }
    return MLMC_OK;
}

mlmc_status mlmc_levels_batch(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoffs,
                              int npayoffs, int M, int L, const uint64_t* N,
                              const uint64_t* offsets, uint64_t seed, mlmc_level_result* out)
{
    if (!ctx) return MLMC_EINVAL;
    if (!payoffs || !N || !out) return fail(ctx, MLMC_EINVAL, "payoffs, N and out must not be NULL");
    if (npayoffs < 1 || npayoffs > kMaxSlots)
        return fail(ctx, MLMC_EINVAL, "npayoffs must be in 1..4");
    mlmc_status st = MLMC_OK;
    for (int k = 0; k < npayoffs && !st; ++k) st = check_level_args(ctx, model, &payoffs[k], L, M, 32);
    if (st) return st;
    if (model->antithetic)
        return fail(ctx, MLMC_EINVAL, "the antithetic estimator runs with per-level launches only");
    if (L >= kMaxLevels) return fail(ctx, MLMC_EINVAL, "L must be < 16");
    for (int i = 0; i < npayoffs * (L + 1); ++i) {
        if (N[i] > (1ull << 40)) return fail(ctx, MLMC_EINVAL, "N too large (max 2^40 per level)");
        if (((offsets ? offsets[i] : 0) + N[i]) >> 56)
            return fail(ctx, MLMC_EINVAL, "path index beyond 2^56");
    }
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    st = ensure_bufs(ctx);
    if (st) return st;
    auto* b = bufs_of(ctx);
    // request: dN and offsets per (slot, level)
    std::memset(b->h_req, 0, sizeof(double) * 2 * kMaxSlots * kMaxLevels);
    for (int k = 0; k < npayoffs; ++k)
        for (int l = 0; l <= L; ++l) {
            b->h_req[k * kMaxLevels + l] = (double)N[k * (L + 1) + l];
            b->h_req[kMaxSlots * kMaxLevels + k * kMaxLevels + l] =
                offsets ? (double)offsets[k * (L + 1) + l] : 0.0;
        }
    fill_desc(ctx, b->h_desc, *model, payoffs, npayoffs, L, M, seed, b->d_req,
              b->d_req + kMaxSlots * kMaxLevels, b->d_acc);
    MLMC_HIP(ctx, hipMemcpyAsync(b->d_req, b->h_req, sizeof(double) * 2 * kMaxSlots * kMaxLevels,
                                 hipMemcpyHostToDevice, ctx->stream));
    st = upload_desc(ctx, b);
    if (st) return st;
    const PersistentShape s = persistent_shape(ctx);
    const int key[5] = {sampler_variant(*model), M, s.block, s.ppt, s.blocks_per_cu};
    if (!b->graph || std::memcmp(key, b->graph_key, sizeof(key)) != 0) {
        if (b->graph) hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        st = capture(ctx, sampler_variant(*model), M, true, nullptr, &b->graph);
        if (st) return st;
        std::memcpy(b->graph_key, key, sizeof(key));
    }
    double fine = 0.0, coarse = 0.0;
    for (int k = 0; k < npayoffs; ++k)
        for (int l = 0; l <= L; ++l) {
            const double nf = std::pow((double)M, (double)l);
            fine += (double)N[k * (L + 1) + l] * nf;
            coarse += l ? (double)N[k * (L + 1) + l] * nf / M : 0.0;
        }
    const int tix = timed_begin(ctx, 16, fine, coarse);
    MLMC_HIP(ctx, hipGraphLaunch(b->graph, ctx->stream));
    timed_end(ctx, tix);
    static_assert(kMaxSlots * kMaxLevels <= kAccSlots, "the folded records fit the host copy");
    LevelAcc* h_acc = ctx->h_acc;
    MLMC_HIP(ctx, hipMemcpyAsync(h_acc, b->d_rec, sizeof(LevelAcc) * kMaxSlots * kMaxLevels,
                                 hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    harvest_timing(ctx);
    uint64_t nonfinite = 0;
    for (int k = 0; k < npayoffs; ++k)
        for (int l = 0; l <= L; ++l) {
            const LevelAcc& r = h_acc[k * kMaxLevels + l];
            mlmc_level_result& o = out[k * (L + 1) + l];
            o.sum_y = r.sum[0];
            o.sum_y2 = r.sum[1];
            o.sum_pf = r.sum[2];
            o.sum_pf2 = r.sum[3];
            o.sum_pc = r.sum[4];
            o.sum_pc2 = r.sum[5];
            const double nf = std::pow((double)M, (double)l);
            o.n = N[k * (L + 1) + l];
            o.cost = (double)o.n * (l ? nf + nf / M : 1.0);
            o.n_nonfinite = r.n_nonfinite;
            nonfinite += r.n_nonfinite;
        }
    if (nonfinite) return fail(ctx, MLMC_ENONFINITE, "non-finite samples left out of the sums");
    return MLMC_OK;
}

}  // extern "C"
