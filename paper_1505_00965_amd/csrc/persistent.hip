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
// by host copies): a batch of levels is a graph captured once and replayed,
// and the adaptive driver's run is two plain launches per iteration (the
// sampler, then one block that absorbs the batch and plans the next).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "context.hpp"
#include "driver.hpp"
#include "driver_dev.hpp"
#include "persistent.hpp"
#include "trace.hpp"

namespace mlmc {

__global__ __launch_bounds__(256) void plan_kernel(const BatchDesc* d)
{
    plan_body(plan_args(d), d->dN, d->offset);
}

// The adaptive run's first kernel when its spread groups are not known to
// hold zeros: a fresh state (n_pilot samples outstanding on levels
// 0..L_min) built in LDS and planned from there (the plan also zeroes the
// dispenser), then the state written out and the spread groups cleared (the
// stores last: nothing waits for them).
__global__ __launch_bounds__(256) void driver_start_kernel(DriverState* st, LevelAcc* spread,
                                                           DriverInit c, const BatchDesc* d)
{
    __shared__ DriverState s;
    const PlanArgs pa = plan_args(d);
    init_state(s, c);   // ends with a barrier
    plan_body(pa, s.dN, s.n);
    constexpr int kWords = sizeof(DriverState) / 8;
    const unsigned long long* w = (const unsigned long long*)&s;
    unsigned long long* dst = (unsigned long long*)st;
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) dst[i] = w[i];
    clear_groups(spread, kMaxLevels - 1);
}

// One iteration's end: sum the spread groups, absorb the batch, re-plan
// (update_state), plan the next batch's items from the new state in LDS,
// then write the state back and clear the groups.  The host reads the
// update count every iteration and the state once, at the end: the mirror
// is written whole by the finishing update only.  Every load goes out at
// the start, none waiting for another: the state (one word per thread), the
// records of every level's spread group (8 waves, levels w and w + 8; the
// groups past the sampled levels hold zeros), the descriptor's plan fields
// and the state's level count and done flag; the stores come last.  A
// finished state has no outstanding samples: the plan its finishing update
// wrote is empty, so a sampler launched after it does nothing, and the
// update launched after it (the host queues exactly one iteration past the
// last) prepares the next run's start instead.
__global__ __launch_bounds__(512) void driver_update_plan_kernel(DriverState* st, DriverState* mirror,
                                                                 LevelAcc* spread, const BatchDesc* d)
{
    constexpr int kWords = sizeof(DriverState) / 8;
    static_assert(kWords <= 512, "one state word per thread");
    static_assert(kMaxLevels == 16 && kSpread == 64, "8 waves, two levels' groups each");
    __shared__ DriverState s;
    __shared__ GroupSums g;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const unsigned long long word =
        threadIdx.x < (unsigned)kWords ? ((const unsigned long long*)st)[threadIdx.x] : 0ull;
    const LevelAcc& r0 = spread[wave * kSpread + lane];
    const LevelAcc& r1 = spread[(wave + 8) * kSpread + lane];
    double y0 = r0.sum[0], q0 = r0.sum[1], c0 = (double)r0.n_nonfinite;
    double y1 = r1.sum[0], q1 = r1.sum[1], c1 = (double)r1.n_nonfinite;
    // the levels the batch sampled: 0..L of the stored state
    const int L0 = __builtin_amdgcn_readfirstlane(st->L);
    const int done = __builtin_amdgcn_readfirstlane(st->done);
    const PlanArgs pa = plan_args(d);
    // only the plan reads the descriptor's fields, at the end: taking them
    // into registers here keeps their loads beside the others
    asm volatile("" ::"s"(pa.L), "s"(pa.M), "s"(pa.nslots), "s"(pa.dim), "s"(pa.split_ok), "s"(pa.num_cu),
                 "s"(pa.resident_blocks), "s"(pa.chunk), "s"(pa.block), "s"(pa.cond_slots), "s"(pa.plan),
                 "s"(pa.head), "s"(pa.split));
    // the sums of each group, in record order as the per-level form folds them
    y0 = wave_sum(y0);
    q0 = wave_sum(q0);
    c0 = wave_sum(c0);
    y1 = wave_sum(y1);
    q1 = wave_sum(q1);
    c1 = wave_sum(c1);
    if (done) {   // block-uniform
        // The update queued past a run's finishing one: the state becomes
        // the fresh state of a next run of this descriptor and the plan its
        // pilot batch (the start kernel's work; the groups already hold
        // zeros), so that run can start with its sampler.  The mirror, which
        // holds the finished run's result, is not touched.
        init_state(s, d->init);   // ends with a barrier
        plan_body(pa, s.dN, s.n);
        if (threadIdx.x < (unsigned)kWords)
            ((unsigned long long*)st)[threadIdx.x] = ((const unsigned long long*)&s)[threadIdx.x];
        return;
    }
    if (lane == 0) {
        g.y[wave] = y0;
        g.y2[wave] = q0;
        g.c[wave] = c0;
        g.y[wave + 8] = y1;
        g.y2[wave + 8] = q1;
        g.c[wave + 8] = c1;
    }
    if (threadIdx.x < (unsigned)kWords) ((unsigned long long*)&s)[threadIdx.x] = word;
    __syncthreads();
    // absorb the groups into the batch records (held at zero between updates)
    if ((int)threadIdx.x <= L0) {
        const int l = (int)threadIdx.x;
        s.batch[l].sum[0] += g.y[l];
        s.batch[l].sum[1] += g.y2[l];
        s.batch[l].n_nonfinite += (unsigned long long)g.c[l];
    }
    __syncthreads();
    update_state(s);   // ends with a barrier
    plan_body(pa, s.dN, s.n);
    publish_state(st, mirror, s, false);
    clear_groups(spread, L0);
}

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

extern template PersistentFn pick_persistent_variant<kGBM>(int, int, int, bool);
extern template PersistentFn pick_persistent_variant<kGBMMil>(int, int, int, bool);
extern template PersistentFn pick_persistent_variant<kHeston>(int, int, int, bool);

// variant: sampler_variant() of the model (GBM Euler, GBM Milstein, Heston);
// payoff: the kind every slot holds, or kAnyPayoff; cv: with the tabulated
// control variate (nullptr where that kernel does not exist).
static PersistentFn pick_persistent(int variant, int M, int ppt, int payoff, bool cv = false)
{
    if (variant == kGBM) return pick_persistent_variant<kGBM>(M, ppt, payoff, cv);
    if (variant == kGBMMil) return pick_persistent_variant<kGBMMil>(M, ppt, payoff, cv);
    return pick_persistent_variant<kHeston>(M, ppt, payoff, cv);
}

// Device buffers of the persistent form, owned by the context.
struct PersistentBufs {
    BatchDesc* d_desc = nullptr;
    BatchDesc* h_desc = nullptr;
    PlanTable* d_plan = nullptr;
    unsigned* d_counters = nullptr;   // head
    LevelAcc* d_acc = nullptr;        // batch spread groups [kMaxSlots][kMaxLevels][kSpread]
    LevelAcc* d_rec = nullptr;        // their folds [kMaxSlots][kMaxLevels]
    unsigned* d_split = nullptr;      // lanes per path [kMaxSlots][kMaxLevels]
    double* d_req = nullptr;          // dN[kMaxSlots][kMaxLevels], offset[...]
    double* h_req = nullptr;
    hipGraphExec_t graph = nullptr;   // cached batch graph
    int graph_key[6] = {-1, -1, -1, -1, -1, -1};
    BatchDesc last_desc;              // the bytes of the last descriptor upload
    // 0: unknown; 1: the device descriptor holds last_desc
    int desc_state = 0;
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
    if (e == hipSuccess) e = hipMalloc(&b->d_plan, sizeof(PlanTable));
    if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(unsigned) * 4);
    // the dispensers start at zero (a driver run's plans leave its own there)
    if (e == hipSuccess) e = hipMemsetAsync(b->d_counters, 0, sizeof(unsigned) * 4, ctx->stream);
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
    if (b->d_desc) hipFree(b->d_desc);
    if (b->h_desc) hipHostFree(b->h_desc);
    if (b->d_plan) hipFree(b->d_plan);
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
// A driver run passes the fresh state's configuration and its own
// dispenser (`head`); a batch passes nullptr and the batch dispenser.
static void fill_desc(mlmc_ctx* ctx, BatchDesc* h, const mlmc_model& m, const mlmc_payoff* p,
                      int np, int L, int M, uint64_t seed, const double* dN, const double* off,
                      LevelAcc* acc, unsigned* head, const DriverInit* init)
{
    auto* b = bufs_of(ctx);
    const PersistentShape s = persistent_shape(ctx);
    std::memset(h, 0, sizeof(*h));
    h->nslots = np;
    h->L = L;
    h->M = M;
    h->dim = m.kind == MLMC_HESTON ? 2 : 1;
    for (int k = 0; k < np; ++k) {
        h->payoff_kind[k] = p[k].kind;
        for (int l = 0; l <= L; ++l) h->params[k][l] = make_step_params<float>(m, p[k], l, M);
    }
    h->seed = seed;
    h->dN = dN;
    h->offset = off;
    h->acc = acc;
    h->plan = b->d_plan;
    h->head = head;
    h->resident_blocks = (unsigned)(ctx->num_cu * s.blocks_per_cu);
    h->chunk = (unsigned)(s.block * s.ppt);
    h->split = b->d_split;
    h->split_ok = m.kind == MLMC_GBM && !m.antithetic;
    h->num_cu = ctx->num_cu;
    h->block = (unsigned)s.block;
    if (init) h->init = *init;
}

// Copy the host descriptor to the device unless the last upload from this
// context carried the same bytes (repeated runs of one problem skip it: a
// driver run passes its seed with each launch, not in the descriptor).
// *uploaded (if given) tells which.
static mlmc_status upload_desc(mlmc_ctx* ctx, PersistentBufs* b, bool* uploaded = nullptr)
{
    if (uploaded) *uploaded = false;
    if (b->desc_state == 1 && std::memcmp(&b->last_desc, b->h_desc, sizeof(BatchDesc)) == 0)
        return MLMC_OK;
    if (uploaded) *uploaded = true;
    b->desc_state = 0;
    MLMC_HIP(ctx, hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice,
                                 ctx->stream));
    std::memcpy(&b->last_desc, b->h_desc, sizeof(BatchDesc));
    b->desc_state = 1;
    return MLMC_OK;
}

// Capture zero -> plan -> persistent -> fold into a graph (payoff: the kind
// of every slot, or kAnyPayoff).
static mlmc_status capture(mlmc_ctx* ctx, int model, int M, int payoff, hipGraphExec_t* out)
{
    auto* b = bufs_of(ctx);
    const PersistentShape s = persistent_shape(ctx);
    hipStream_t cs;
    MLMC_HIP(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = zero_records(b->d_acc, kMaxSlots * kMaxLevels * kSpread, cs);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(256), 0, cs, (const BatchDesc*)b->d_desc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        // the seed from the descriptor (uploaded per batch), the plan from plan_kernel
        hipLaunchKernelGGL(pick_persistent(model, M, s.ppt, payoff), dim3(ctx->num_cu * s.blocks_per_cu),
                           dim3(s.block), 0, cs, (const BatchDesc*)b->d_desc, (uint64_t)0, 0u);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fold_groups_kernel, dim3(kMaxSlots * kMaxLevels), dim3(kSpread), 0, cs,
                           b->d_acc, b->d_rec);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(ctx, e, "persistent graph capture");
    return MLMC_OK;
}

// mlmc_run with persistent = 1: the start kernel (fresh state, pilot plan),
// then per driver iteration the all-levels sampler and the update-and-plan
// block, as plain launches on the context's stream.
mlmc_status run_persistent(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p,
                           const mlmc_run_opts& o, DriverState* d_st, DriverState* h_st,
                           const DriverInit& init, bool prepared)
{
    if (o.precision != 32) return fail(ctx, MLMC_EINVAL, "the persistent form runs fp32 paths");
    if (o.cv) {
        if (!cv_tabulated(o.cv))
            return fail(ctx, MLMC_EINVAL,
                        "the device-planned form takes the tabulated control variate (mlmc_cv_set_tabulated)");
        if (m.scheme != MLMC_EULER || m.antithetic)
            return fail(ctx, MLMC_EINVAL, "the control variate runs with plain Euler paths");
        if (p.kind == MLMC_DIGITAL_COND)
            return fail(ctx, MLMC_EINVAL, "the control variate takes the four plain payoffs");
        if (cv_in_dim(o.cv) != (m.kind == MLMC_HESTON ? 3 : 2))
            return fail(ctx, MLMC_EINVAL, "network inputs do not match the model (2: GBM, 3: Heston)");
    }
    mlmc_status st = ensure_bufs(ctx);
    if (st) return st;
    auto* b = bufs_of(ctx);
    // the seed goes in with each launch: runs of one problem share the
    // descriptor's bytes and upload it once.  Driver runs have a dispenser
    // of their own, which their plans leave at zero.
    fill_desc(ctx, b->h_desc, m, &p, 1, o.L_max, o.M, 0, d_st->dN, d_st->n, ctx->d_drv_spread,
              b->d_counters + 1, &init);
    size_t lds = 0;
    if (o.cv) {
        int max_nf = 1;
        for (int l = 0; l < o.L_max; ++l) max_nf *= o.M;
        const hipError_t e = cv_table_view(o.cv, m, ctx->stream, max_nf, &b->h_desc->cv_table,
                                           &b->h_desc->cv_spec, &b->h_desc->cv_phi0, &lds);
        if (e != hipSuccess) return hip_fail(ctx, e, "control-variate table");
        b->h_desc->cv_levels = o.cv_levels;
    }
    bool uploaded = false;
    st = upload_desc(ctx, b, &uploaded);
    if (st) return st;
    const PersistentShape s = persistent_shape(ctx);
    const auto sampler = pick_persistent(sampler_variant(m), o.M, s.ppt, p.kind, o.cv != nullptr);
    if (!sampler) return fail(ctx, MLMC_EINVAL, "no persistent sampler for this model and payoff");
    const dim3 grid(ctx->num_cu * s.blocks_per_cu), block(s.block);
    const BatchDesc* d = b->d_desc;
    DriverState* mirror = (DriverState*)ctx->h_drv_dev;
    // prepared: the context's last call was a device-planned run that ended
    // normally, so the update queued past its end has built a fresh state
    // and planned its pilot batch, and its updates left the spread groups at
    // zero; if the descriptor is that run's, this run starts with its
    // sampler.  Otherwise the start kernel comes first.
    if (!(prepared && !uploaded)) {
        hipLaunchKernelGGL(driver_start_kernel, dim3(1), dim3(256), 0, ctx->stream, d_st,
                           ctx->d_drv_spread, init, d);
        MLMC_HIP(ctx, hipGetLastError());
    }
    // Iteration k + 1 is enqueued before the host waits for iteration k's
    // update: its sampler reads the items that update planned, so the GPU
    // runs the iterations back to back while the host reads the mirror.  The
    // one iteration past the last update finds an empty plan and a finished
    // state and does nothing.
    int first_tix = -1;
    for (int it = 0;; ++it) {
        if (it > h_st->max_iterations + 1)
            return fail(ctx, MLMC_EDEVICE, "driver state did not reach the host");
        const TraceRange iter_range("mlmc_run driver iteration (device-planned)");
        for (int k = it ? 1 : 0; k < 2; ++k) {
            // the sampler stamps slot 16, the update-and-plan block slot 17
            hipEvent_t t0, t1;
            timed_kernel(ctx, 16, 0.0, 0.0, &t0, &t1);
            if (first_tix < 0 && t0) first_tix = (int)ctx->pending.size() - 1;
            const unsigned flags = kSeedArg;
            if (t0) hipExtLaunchKernelGGL(sampler, grid, block, lds, ctx->stream, t0, t1, 0, d, o.seed, flags);
            else hipLaunchKernelGGL(sampler, grid, block, lds, ctx->stream, d, o.seed, flags);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) {
                timed_kernel(ctx, 17, 0.0, 0.0, &t0, &t1);
                if (t0)
                    hipExtLaunchKernelGGL(driver_update_plan_kernel, dim3(1), dim3(512), 0, ctx->stream,
                                          t0, t1, 0, d_st, mirror, ctx->d_drv_spread, d);
                else
                    hipLaunchKernelGGL(driver_update_plan_kernel, dim3(1), dim3(512), 0, ctx->stream,
                                       d_st, mirror, ctx->d_drv_spread, d);
                e = hipGetLastError();
            }
            if (e != hipSuccess) return hip_fail(ctx, e, "persistent iteration");
        }
        // the update kernel also writes the host mirror h_st
        const hipError_t e = wait_update(ctx->stream, h_st, (unsigned long long)it + 1);
        if (e != hipSuccess) return hip_fail(ctx, e, "persistent iteration");
        // the flag comes in the word that publishes the update, so a mirror
        // seen done is complete; later updates leave it as it is
        if (mirror_done(h_st)) break;
    }
    // the update queued past the last one prepares the next run's start
    ctx->drv_pilot_ready = true;
    // the iteration past the last update may still run: the result is read
    // from the mirror; stamped launches are read once finished (harvest_ready
    // now, the rest by a later harvest), the run does not wait for them
    if (ctx->pending.empty()) return MLMC_OK;
    if (first_tix >= 0) {
        // the launches' path steps are known only as a whole: every sampled
        // batch is absorbed into n_l, so they are charged to the run's first
        // stamped sampler launch
        double fine = 0.0, coarse = 0.0;
        for (int l = 0; l <= h_st->L; ++l) {
            const double nf = std::pow((double)o.M, (double)l);
            fine += h_st->n[l] * nf;
            coarse += l ? h_st->n[l] * nf / o.M : 0.0;
        }
        ctx->pending[first_tix].fine_steps = fine;
        ctx->pending[first_tix].coarse_steps = coarse;
    }
    harvest_ready(ctx);
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
        b->graph = nullptr;
        b->graph_key[0] = -1;
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
    // a batch rewrites the plan table: a driver run's prepared start is gone
    ctx->drv_pilot_ready = false;
    fill_desc(ctx, b->h_desc, *model, payoffs, npayoffs, L, M, seed, b->d_req,
              b->d_req + kMaxSlots * kMaxLevels, b->d_acc, b->d_counters, nullptr);
    MLMC_HIP(ctx, hipMemcpyAsync(b->d_req, b->h_req, sizeof(double) * 2 * kMaxSlots * kMaxLevels,
                                 hipMemcpyHostToDevice, ctx->stream));
    st = upload_desc(ctx, b);
    if (st) return st;
    const PersistentShape s = persistent_shape(ctx);
    // one payoff kind in every slot: the kernel holds that payoff's code only
    int payoff = payoffs[0].kind;
    for (int k = 1; k < npayoffs; ++k)
        if (payoffs[k].kind != payoff) payoff = kAnyPayoff;
    const int key[6] = {sampler_variant(*model), M, s.block, s.ppt, s.blocks_per_cu, payoff};
    if (!b->graph || std::memcmp(key, b->graph_key, sizeof(key)) != 0) {
        if (b->graph) hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        st = capture(ctx, sampler_variant(*model), M, payoff, &b->graph);
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
