// Persistent all-levels sampler: the batch descriptor, the work items and
// the sampler kernel (its plan and host side are in persistent.hip).  The
// kernel is instantiated per model variant in persistent_<variant>.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "cv_tab.hpp"
#include "driver.hpp"
#include "level.hpp"
#include "sampler_impl.hpp"

namespace mlmc {

constexpr int kMaxSlots = 4;          // payoffs per batch
constexpr int kPairs = kMaxSlots * kMaxLevels;
constexpr int kItemsPerBlock = 4;     // target items per resident block
constexpr unsigned kItemsPerPair = 1024;

struct WorkItem {
    uint64_t first;     // first sample index of the range
    uint32_t n;         // number of samples
    uint16_t level;
    uint8_t slot;       // payoff slot
    uint8_t pad;
};

// The plan of one launch: the (slot, level) pairs with outstanding samples,
// in processing order; pair q owns items start[q] .. start[q+1] - 1, which
// cut [first[q], first[q] + left[q]) at base[q] + i per[q] (base[q] <=
// first[q]: the first and last pieces may be shorter).  Items are decoded
// from it by the sampler, not stored.
struct PlanTable {
    uint64_t first[kPairs], left[kPairs], per[kPairs], base[kPairs];
    unsigned start[kPairs + 1];
    int npairs;
    uint8_t slot[kPairs], level[kPairs];
    uint32_t pad[1];
};
static_assert(sizeof(PlanTable) % 8 == 0, "copied in 8-byte words");

// Device-resident batch description (rewritten before each launch).
struct BatchDesc {
    int nslots, L, M;
    int dim;                          // Brownian dimension: 1 (GBM), 2 (Heston)
    int payoff_kind[kMaxSlots];
    StepParams<float> params[kMaxSlots][kMaxLevels];
    uint64_t seed;
    // outstanding samples and their first index, per (slot, level); for the
    // driver these alias DriverState::dN / n (slot 0 only)
    const double* dN;
    const double* offset;
    LevelAcc* acc;                    // spread groups [slot][level][kSpread]
    PlanTable* plan;                  // written by the plan, read by the sampler
    unsigned* head;                   // dispenser of the items past the first gridDim.x
    unsigned resident_blocks;         // grid size of the sampler
    unsigned chunk;                   // blockDim * PPT of the sampler
    unsigned block;                   // blockDim of the sampler
    unsigned* split;                  // lanes per path per (slot, level), set by the plan
    int split_ok;                     // the model's paths are linear in their start (GBM)
    int num_cu;
    // the tabulated control variate of a driver run (the sampler kernel
    // compiled with it): its table and grid, phi(0, S0) from the table, and
    // the levels it applies to (l < cv_levels, or all for 0)
    const float* cv_table;
    TableSpec cv_spec;
    const float* cv_phi0;
    int cv_levels;
    // a driver run: the configuration of a fresh state (the update that
    // finds a run finished builds the next run's from it)
    DriverInit init;
};

// A batch whose slots may hold different payoff kinds.
constexpr int kAnyPayoff = -1;

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
        // one or two steps: samples share generator blocks (two-step levels
        // exist for M = 2 only: the other code is not compiled for M = 4)
        constexpr int D = one_factor(MODEL) ? 1 : 2;
        const int q = M == 2 ? 4 / (a.nf * D) : 4 / D;
        const uint64_t nblk = short_blocks(a.offset, a.N, q);
        const uint64_t chunk = (uint64_t)blockDim.x * PPT;
        const FullChunks f = full_chunks(a.offset, a.N, q, chunk);
        const uint32_t lo = __builtin_amdgcn_readfirstlane(f.lo), hi = __builtin_amdgcn_readfirstlane(f.hi);
        // one counter segment: chunk indices fit 32 bits (a scalar loop test)
        const uint32_t nch = __builtin_amdgcn_readfirstlane((uint32_t)((nblk + chunk - 1) / chunk));
        for (uint32_t c = 0; c < nch; ++c) {
            const uint64_t base = (uint64_t)c * chunk;
            const bool full = c >= lo && c < hi;
            if (M != 2 || a.nf == 1)
                process_short<MODEL, PAYOFF, float, 1, M, PPT, false>(a, base, full, sums, nonfinite);
            else
                process_short<MODEL, PAYOFF, float, 2, M, PPT, false>(a, base, full, sums, nonfinite);
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

// The samples [a.offset, a.offset + a.N) of one item part of a level >= 1
// with the tabulated control variate (the level's rows in LDS, tv): the
// per-level kernels' paths (split GBM paths, two-step samples at M = 2, or
// up to two samples per lane).
template <int MODEL, int PAYOFF, int M, int PPT>
__device__ __forceinline__ void run_range_tab(const LevelArgs<float>& a, const TabView& tv,
                                              double (&sums)[kNumSums], unsigned& nonfinite)
{
    if constexpr (MODEL == kGBM) {
        if (a.split > 1) {
            const uint64_t pass = blockDim.x / a.split;
            for (uint64_t base = 0; base < a.N; base += pass)
                process_split_tab<PAYOFF, M>(a, base, tv, sums, nonfinite);
            return;
        }
    }
    if (a.nf < 4) {
        if constexpr (M == 2) {
            for (uint64_t base = 0; base < a.N; base += blockDim.x)
                process_short_tab<MODEL, PAYOFF, M>(a, base, tv, sums, nonfinite);
        }
        return;
    }
    constexpr int TP = PPT > 2 ? 2 : PPT;
    const uint64_t chunk = (uint64_t)blockDim.x * TP;
    for (uint64_t base = 0; base < a.N; base += chunk)
        process_chunk_tab<MODEL, PAYOFF, M, TP>(a, base, tv, sums, nonfinite);
}

// A copy of v that the compiler knows to be the same in every lane (it
// must be): each 32-bit word read from the first active lane, so the item
// and its parameters live in scalar registers, as a launch's arguments do.
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v)
{
    static_assert(sizeof(T) % 4 == 0, "copied in 32-bit words");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

// One item.  CV: the kernel carries the tabulated control variate; an item
// of a level it applies to takes phi(0, S0) (level 0) or the level's table
// rows, copied into s_tab unless the block's previous item left them there
// (tab_level, block-uniform; items are separated by barriers).
template <int MODEL, int PAYOFF, int M, int PPT, bool CV>
__device__ __forceinline__ void run_item(const BatchDesc* d, uint64_t seed, const WorkItem& w, double (&sums)[kNumSums],
                                         unsigned& nonfinite, float* s_tab, int& tab_level)
{
    LevelArgs<float> a;
    a.P = wave_uniform(d->params[w.slot][w.level]);
    a.seed = seed;
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
    a.split = __builtin_amdgcn_readfirstlane(d->split[w.slot * kMaxLevels + w.level]);
    bool tab = false;
    TabView tv{};
    if constexpr (CV) {
        const int cl = __builtin_amdgcn_readfirstlane(d->cv_levels);
        if (cl <= 0 || (int)w.level < cl) {
            if (w.level == 0) {
                a.phi0 = d->cv_phi0;
            } else {
                tab = true;
                const TableSpec t = wave_uniform(d->cv_spec);
                if (tab_level != (int)w.level) {
                    tv = load_level_table(s_tab, d->cv_table, t, nf);   // ends with a barrier
                    tab_level = w.level;
                } else {
                    const int lr = nf < t.rows ? nf : t.rows;
                    tv = TabView{s_tab, t, lr, nf};
                }
            }
        }
    }
    constexpr int D = one_factor(MODEL) ? 1 : 2;
    // one pass per part of the item whose generator units share counter word 2
    const uint64_t q = samples_per_unit(nf, D), end = w.first + w.n;
    for (uint64_t first = w.first; first < end;) {
        const uint64_t stop = counter_segment_end(first, end, q);
        a.offset = first;
        a.N = stop - first;
        set_counter_words(a, D);
        if (CV && tab) run_range_tab<MODEL, PAYOFF, M, PPT>(a, tv, sums, nonfinite);
        else run_range<MODEL, PAYOFF, M, PPT>(a, sums, nonfinite);
        first = stop;
    }
}

// What the plan reads of the descriptor besides the request: loaded at a
// kernel's start, so the loads overlap the kernel's other reads.
struct PlanArgs {
    int L, M, nslots, dim, split_ok, num_cu;
    unsigned resident_blocks, chunk, block;
    unsigned cond_slots;              // bit k: slot k holds the conditional digital
    PlanTable* plan;
    unsigned* head;
    unsigned* split;
};

__device__ __forceinline__ PlanArgs plan_args(const BatchDesc* d)
{
    PlanArgs a;
    a.L = d->L;
    a.M = d->M;
    a.nslots = d->nslots;
    a.dim = d->dim;
    a.split_ok = d->split_ok;
    a.num_cu = d->num_cu;
    a.resident_blocks = d->resident_blocks;
    a.chunk = d->chunk;
    a.block = d->block;
    a.cond_slots = 0;
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k) a.cond_slots |= d->payoff_kind[k] == kDigitalCond ? 1u << k : 0u;
    a.plan = d->plan;
    a.head = d->head;
    a.split = d->split;
    return a;
}

// ceil(a / b) for a < 2^53, b > 0: the fp64 quotient is within one of it.
__device__ __forceinline__ uint64_t ceil_div_u53(uint64_t a, uint64_t b)
{
    uint64_t q = (uint64_t)ceil((double)a / (double)b);
    if (q * b < a) ++q;
    else if (q && (q - 1) * b >= a) --q;
    return q;
}

// Plan: the first wave sizes the (slot, level) pairs, one lane each, in
// processing order (deepest level first, then slot), so the per-pair
// arithmetic runs side by side; a wave scan gives each pair its first item,
// and each lane writes its pair's row of the plan table (the sampler decodes
// the items from it).  dN and off: the outstanding samples and their first
// index per (slot, level) (device memory, or the driver state in LDS).  Only
// the first wave works; every thread of the block may call it.  Block sizes
// and samples per lane are powers of two (the launch shape's rule), and so
// are the sampler's chunks and split passes: they are cut with masks.
__device__ __forceinline__ void plan_body(const PlanArgs& a, const double* dN, const double* off)
{
    static_assert(kPairs == 64, "one lane of the first wave per (slot, level) pair");
    if (threadIdx.x >= 64) return;
    const int L = a.L, M = a.M, nslots = a.nslots;
    const int p = (int)threadIdx.x;
    const bool valid = p < (L + 1) * nslots;
    const int l = valid ? L - p / nslots : 0, s = valid ? p % nslots : 0;
    double nf = 1.0;
    for (int i = 0; i < l; ++i) nf *= M;   // M^l, exact
    const double per = nf + (l ? nf / M : 0.0);
    const double dn = valid ? dN[s * kMaxLevels + l] : 0.0;
    // samples x steps over the batch (lane 0's sum: the rotations leave
    // other lanes with other association orders)
    const double total = __shfl(wave_sum(valid ? dn * per : 0.0), 0);
    const double target = total / ((double)a.resident_blocks * kItemsPerBlock);
    const uint64_t left = (uint64_t)dn;
    const uint64_t first = valid ? (uint64_t)off[s * kMaxLevels + l] : 0;
    uint64_t base = first;
    unsigned items = 0;
    uint64_t per_item = 0;
    if (valid) {
        // lanes per path: the per-level launch's rule on the same count
        const uint32_t G = split_lanes((int)nf, left, a.num_cu, a.split_ok && !((a.cond_slots >> s) & 1u));
        a.split[s * kMaxLevels + l] = G;
        if (left) {
            uint64_t paths = (uint64_t)(target / per);
            // samples of one chunk of the sampler: block x ppt samples, or on
            // one- and two-step levels block x ppt generator blocks of q
            const uint64_t unit = (uint64_t)a.chunk * (nf < 4 ? (uint64_t)(4 / ((int)nf * a.dim)) : 1ull);
            if (G > 1) {
                // split paths: whole block passes of block / G paths
                const uint64_t pass = a.block / G;
                paths = paths < pass ? pass : paths & ~(pass - 1);
            } else if (paths >= unit) {
                paths &= ~(unit - 1);                    // whole chunks where possible
            } else {
                // one sample per lane, or one whole chunk, whichever is nearer
                paths = 2 * paths >= a.block + unit ? unit : a.block;
            }
            if (paths > (1ull << 31)) paths = 1ull << 31;   // item sizes fit 32 bits
            // at most kItemsPerPair items per pair (one more when cut on the
            // chunk grid below): item indices stay small
            const uint64_t min_items = (left + kItemsPerPair - 1) / kItemsPerPair;
            per_item = paths > min_items ? paths : min_items;
            if (G == 1 && per_item > a.block) {
                // whole chunks (the sampler simulates a whole chunk, the
                // samples past the item's end included), cut on a grid of
                // whole chunks from the pair's first sample rounded down:
                // every piece but the pair's first and last then fills all
                // its chunks (on one- and two-step levels a partial chunk
                // also takes per-sample range checks)
                per_item = (per_item + unit - 1) & ~(unit - 1);
                base = first & ~(unit - 1);
            }
            if (per_item > (1ull << 31)) per_item = (1ull << 31) & ~(unit - 1);
            items = (unsigned)ceil_div_u53(first + left - base, per_item);
        }
    }
    // inclusive scan of the item counts over the lanes (pair order)
    unsigned incl = items;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
        const unsigned v = __shfl_up(incl, k);
        if (p >= k) incl += v;
    }
    // pairs with samples, packed in order
    const uint64_t active = __ballot(items > 0);
    const int rank = __popcll(active & ((1ull << p) - 1ull));
    PlanTable* t = a.plan;
    if (items) {
        t->first[rank] = first;
        t->left[rank] = left;
        t->per[rank] = per_item;
        t->base[rank] = base;
        t->slot[rank] = (uint8_t)s;
        t->level[rank] = (uint8_t)l;
        t->start[rank] = incl - items;
    }
    if (p == 63) {
        const int np = __popcll(active);
        t->start[np] = incl;
        t->npairs = np;
        if (a.head) *a.head = 0;
    }
}

// Item `it` of the plan (block-uniform).
__device__ __forceinline__ WorkItem plan_item(const PlanTable& t, unsigned it)
{
    int q = 0;
    while (q + 1 < t.npairs && t.start[q + 1] <= it) ++q;
    const uint64_t lo = t.base[q] + (uint64_t)(it - t.start[q]) * t.per[q];
    const uint64_t hi = lo + t.per[q], end = t.first[q] + t.left[q];
    WorkItem w;
    w.first = lo > t.first[q] ? lo : t.first[q];
    w.n = (uint32_t)((hi < end ? hi : end) - w.first);
    w.level = t.level[q];
    w.slot = t.slot[q];
    w.pad = 0;
    return w;
}

// Launch flags of the sampler.
constexpr unsigned kSeedArg = 1;   // the seed is the launch's argument (else the descriptor's)

// Block b takes item b first; later items come from the dispenser until
// none are left, so a launch with no more items than blocks (an empty one
// included) makes no atomics on it.  Each item ends with a block reduction
// into its (payoff, level) spread group.
template <int MODEL, int M, int PPT, int PAYOFF, bool CV>
__device__ __forceinline__ void sample_items(const BatchDesc* d, float* s_tab, uint64_t seed_arg,
                                             unsigned flags)
{
    __shared__ unsigned s_item;
    // the plan in LDS: each item is decoded by a short search over its pairs
    __shared__ PlanTable s_plan;
    {
        const unsigned long long* src = (const unsigned long long*)d->plan;
        unsigned long long* dst = (unsigned long long*)&s_plan;
        for (int i = threadIdx.x; i < (int)(sizeof(PlanTable) / 8); i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const uint64_t seed = (flags & kSeedArg) ? seed_arg : d->seed;
    int tab_level = -1;
    const unsigned count = __builtin_amdgcn_readfirstlane(s_plan.start[s_plan.npairs]);
    for (unsigned it = blockIdx.x; it < count;) {   // block-uniform
        const WorkItem w = wave_uniform(plan_item(s_plan, it));
        double sums[kNumSums] = {0, 0, 0, 0, 0, 0};
        unsigned nonfinite = 0;
        if constexpr (PAYOFF == kAnyPayoff) {
            switch (d->payoff_kind[w.slot]) {
            case kCall: run_item<MODEL, kCall, M, PPT, false>(d, seed, w, sums, nonfinite, s_tab, tab_level); break;
            case kAsian: run_item<MODEL, kAsian, M, PPT, false>(d, seed, w, sums, nonfinite, s_tab, tab_level); break;
            case kLookback:
                run_item<MODEL, kLookback, M, PPT, false>(d, seed, w, sums, nonfinite, s_tab, tab_level);
                break;
            case kDigitalCond:
                run_item<MODEL, kDigitalCond, M, PPT, false>(d, seed, w, sums, nonfinite, s_tab, tab_level);
                break;
            default: run_item<MODEL, kDigital, M, PPT, false>(d, seed, w, sums, nonfinite, s_tab, tab_level); break;
            }
        } else {
            run_item<MODEL, PAYOFF, M, PPT, CV>(d, seed, w, sums, nonfinite, s_tab, tab_level);
        }
        if (w.level == 0) copy_y_sums(sums);
        block_reduce_add(sums, nonfinite, &d->acc[(w.slot * kMaxLevels + w.level) * kSpread +
                                                  (blockIdx.x & (kSpread - 1))]);
        if (count <= gridDim.x) break;
        if (threadIdx.x == 0) s_item = gridDim.x + atomicAdd(d->head, 1u);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
    }
}

// PAYOFF: one payoff kind for every slot of the batch, or kAnyPayoff (each
// item's slot names it; the kernel then holds every payoff's code and the
// registers of the largest).  CV: with the tabulated control variate (one
// payoff, Euler paths; launched with the deepest level's table rows of
// dynamic LDS).
template <int MODEL, int M, int PPT, int PAYOFF, bool CV>
__global__ __launch_bounds__(1024) void persistent_kernel(const BatchDesc* d, uint64_t seed, unsigned flags)
{
    extern __shared__ __attribute__((aligned(16))) float s_tab[];
    sample_items<MODEL, M, PPT, PAYOFF, CV>(d, s_tab, seed, flags);
}

using PersistentFn = void (*)(const BatchDesc*, uint64_t, unsigned);

template <int MODEL, int M, int PPT>
PersistentFn pick_persistent_payoff(int payoff, bool cv)
{
    if (cv) {
        // the control variate runs with Euler paths and the four plain payoffs
        if constexpr (MODEL != kGBMMil) {
            switch (payoff) {
            case kCall: return persistent_kernel<MODEL, M, PPT, kCall, true>;
            case kAsian: return persistent_kernel<MODEL, M, PPT, kAsian, true>;
            case kLookback: return persistent_kernel<MODEL, M, PPT, kLookback, true>;
            case kDigital: return persistent_kernel<MODEL, M, PPT, kDigital, true>;
            default: return nullptr;
            }
        }
        return nullptr;
    }
    switch (payoff) {
    case kCall: return persistent_kernel<MODEL, M, PPT, kCall, false>;
    case kAsian: return persistent_kernel<MODEL, M, PPT, kAsian, false>;
    case kLookback: return persistent_kernel<MODEL, M, PPT, kLookback, false>;
    case kDigital: return persistent_kernel<MODEL, M, PPT, kDigital, false>;
    case kDigitalCond: return persistent_kernel<MODEL, M, PPT, kDigitalCond, false>;
    default: return persistent_kernel<MODEL, M, PPT, kAnyPayoff, false>;
    }
}

// The sampler of one model variant for (M, samples per lane, payoff kind or
// kAnyPayoff, with the tabulated control variate or not); nullptr for a
// combination that does not exist.  Defined here, instantiated once per
// variant.
template <int MODEL>
PersistentFn pick_persistent_variant(int M, int ppt, int payoff, bool cv)
{
    if (M == 2) {
        switch (ppt) {
        case 1: return pick_persistent_payoff<MODEL, 2, 1>(payoff, cv);
        case 2: return pick_persistent_payoff<MODEL, 2, 2>(payoff, cv);
        default: return pick_persistent_payoff<MODEL, 2, 4>(payoff, cv);
        }
    }
    switch (ppt) {
    case 1: return pick_persistent_payoff<MODEL, 4, 1>(payoff, cv);
    case 2: return pick_persistent_payoff<MODEL, 4, 2>(payoff, cv);
    default: return pick_persistent_payoff<MODEL, 4, 4>(payoff, cv);
    }
}
}  // namespace mlmc
