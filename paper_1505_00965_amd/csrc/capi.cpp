// C ABI: context management and the per-level entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "context.hpp"

namespace mlmc {

mlmc_status fail(mlmc_ctx* ctx, mlmc_status st, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

mlmc_status hip_fail(mlmc_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, MLMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static int level_steps(int l, int M)
{
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    return nf;
}

const char* level_args_error(const mlmc_model* m, const mlmc_payoff* p, int l, int M, int precision)
{
    if (!m || !p) return "model and payoff must not be NULL";
    if (m->kind != MLMC_GBM && m->kind != MLMC_HESTON) return "unknown model kind";
    if (p->kind < MLMC_CALL || p->kind > MLMC_DIGITAL_COND) return "unknown payoff kind";
    if (M != 2 && M != 4) return "M must be 2 or 4";
    if (l < 0) return "level must be >= 0";
    if ((M == 2 && l > 18) || (M == 4 && l > 9)) return "level too deep: at most 262144 fine steps";
    if (precision != 32 && precision != 64) return "precision must be 32 or 64";
    if (!(m->T > 0) || !(m->S0 > 0) || !std::isfinite(m->r))
        return "model needs T > 0, S0 > 0 and finite r";
    if (m->kind == MLMC_GBM && !(m->sigma >= 0)) return "GBM needs sigma >= 0";
    if (m->kind == MLMC_HESTON &&
        (!(m->rho >= -1 && m->rho <= 1) || !(m->xi >= 0) || !(m->theta >= 0) || !(m->v0 >= 0)))
        return "Heston needs |rho| <= 1 and xi, theta, v0 >= 0";
    if (m->scheme != MLMC_EULER && m->scheme != MLMC_MILSTEIN) return "unknown scheme";
    if (m->scheme == MLMC_MILSTEIN && m->kind != MLMC_GBM)
        return "the Milstein scheme is implemented for GBM only";
    if (m->antithetic != 0 && m->antithetic != 1) return "antithetic must be 0 or 1";
    return nullptr;
}

mlmc_status check_level_args(mlmc_ctx* ctx, const mlmc_model* m, const mlmc_payoff* p, int l, int M,
                             int precision)
{
    if (!ctx) return MLMC_EINVAL;
    const char* why = level_args_error(m, p, l, M, precision);
    return why ? fail(ctx, MLMC_EINVAL, why) : MLMC_OK;
}

// Path steps per sample of level l: n_f + n_c (2 n_f + n_c with the twin).
double level_cost(const mlmc_model& m, int l, int M)
{
    if (l == 0) return 1.0;
    const double nf = std::pow((double)M, (double)l);
    return (m.antithetic ? 2.0 : 1.0) * nf + nf / M;
}

// Split paths (process_split) exist for fp32 GBM paths (Euler or Milstein)
// of the four plain payoffs without the antithetic twin.
static bool split_eligible(const mlmc_model& m, const mlmc_payoff& p, int precision)
{
    return precision == 32 && m.kind == MLMC_GBM && !m.antithetic && p.kind != MLMC_DIGITAL_COND;
}

LaunchShape choose_shape(const mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l,
                         int M, int precision, uint64_t N, uint64_t n_call)
{
    int tb = 0, tp = 0;
    if (ctx->launch_block || !tuned_shape(ctx, m, p.kind, precision, M, l, &tb, &tp)) tb = tp = 0;
    LaunchShape s = default_shape(m, p, l, M, precision, N, n_call, ctx->num_cu, ctx->launch_block,
                                  ctx->launch_ppt, tb, tp);
    s.num_cu = ctx->num_cu;
    return s;
}

LaunchShape default_shape(const mlmc_model& m, const mlmc_payoff& p, int l, int M, int precision,
                          uint64_t N, uint64_t n_call, int num_cu, int fixed_block, int fixed_ppt,
                          int tuned_block, int tuned_ppt)
{
    LaunchShape s;
    s.block = fixed_block ? fixed_block : 256;
    s.ppt = precision == 64 ? 1 : (fixed_ppt ? fixed_ppt : 2);
    if (!fixed_block && tuned_block) {
        s.block = tuned_block;
        s.ppt = tuned_ppt;
    }
    if (!fixed_block) {
        // few samples: fewer paths per thread so that more lanes take part
        // (the tuner measures device-filling counts, so its ppt is for those)
        const uint64_t lanes = (N + s.ppt - 1) / s.ppt;
        if (lanes < (uint64_t)num_cu * 256) s.ppt = 1;
    }
    const int nf = level_steps(l, M);
    uint64_t units = N;   // samples, or generator blocks for one/two-step levels
    if (nf < 4) {
        const int q = 4 / (nf * (m.kind == MLMC_HESTON ? 2 : 1));
        units = (N + q - 1) / q + 1;
        if (s.ppt > 2) s.ppt = 2;
    }
    if (m.antithetic && l > 0 && s.ppt > 2) s.ppt = 2;   // the twin doubles the path state
    // GBM levels whose paths cannot fill the device: several lanes per path
    s.split = split_lanes(nf, n_call ? n_call : N, num_cu, split_eligible(m, p, precision));
    if (s.split > 1) {
        s.ppt = 1;
        units = N;   // paths, block / split per block at a time
    } else if (!fixed_block) {
        // a tuned shape is measured at device-filling counts: for a smaller
        // launch halve the samples per lane, then the block, until the launch
        // has a block per compute unit and two waves per SIMD (or is 64 x 1)
        for (;;) {
            const uint64_t c = (uint64_t)s.block * s.ppt, blocks = (units + c - 1) / c;
            if ((blocks >= (uint64_t)num_cu && blocks * (uint64_t)(s.block / 64) >= 8ull * num_cu) ||
                (s.ppt == 1 && s.block == 64))
                break;
            if (s.ppt > 1) s.ppt /= 2;
            else s.block /= 2;
        }
    }
    const uint64_t chunk = s.split > 1 ? (uint64_t)s.block / s.split : (uint64_t)s.block * s.ppt;
    const uint64_t chunks = (units + chunk - 1) / chunk;
    const uint64_t cap = (uint64_t)num_cu * (2048 / s.block);
    s.grid = (int)std::max<uint64_t>(1, std::min(chunks, cap));
    s.num_cu = 0;   // no residency cap unless the caller sets it
    return s;
}

__global__ void zero_records_kernel(LevelAcc* acc, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        for (int k = 0; k < kNumSums; ++k) acc[i].sum[k] = 0.0;
        acc[i].n_nonfinite = 0;
        acc[i].pad = 0;
    }
}

hipError_t zero_records(LevelAcc* acc, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_records_kernel, dim3((n + 63) / 64), dim3(64), 0, st, acc, n);
    return hipGetLastError();
}

template <typename Real>
static LevelArgs<Real> make_args(const mlmc_model& m, const mlmc_payoff& p, int l, int M, uint64_t N,
                                 uint64_t seed, uint64_t offset, uint32_t stream, int coupled,
                                 LevelAcc* acc, double* d_pf, double* d_pc)
{
    LevelArgs<Real> a;
    a.P = make_step_params<Real>(m, p, l, M);
    a.seed = seed;
    a.offset = offset;
    a.N = N;
    a.l = l;
    a.nf = level_steps(l, M);
    a.ngroups = (uint32_t)((a.nf + 3) / 4);
    a.stream = stream;
    a.acc = acc;
    a.pf_out = d_pf;
    a.pc_out = d_pc;
    a.coupled = coupled;
    a.phi0 = nullptr;
    return a;
}


static hipEvent_t pool_event(mlmc_ctx* ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Timing on for this launch of the slot: its bit is set and, with a stride
// k, it is the first, (k+1)-th, (2k+1)-th ... launch since the mask was set.
static bool time_this(mlmc_ctx* ctx, int slot)
{
    if (ctx->timing_paused || !(ctx->timing >> slot & 1u)) return false;
    return ctx->timing_seen[slot]++ % ctx->timing_stride == 0;
}

int timed_begin(mlmc_ctx* ctx, int slot, double fine_steps, double coarse_steps)
{
    if (!time_this(ctx, slot)) return -1;
    mlmc_ctx::Timed t;
    t.start = pool_event(ctx);
    t.stop = pool_event(ctx);
    if (!t.start || !t.stop) return -1;
    t.slot = slot;
    t.fine_steps = fine_steps;
    t.coarse_steps = coarse_steps;
    hipEventRecord(t.start, ctx->stream);
    ctx->pending.push_back(t);
    return (int)ctx->pending.size() - 1;
}

void timed_kernel(mlmc_ctx* ctx, int slot, double fine_steps, double coarse_steps,
                  hipEvent_t* start, hipEvent_t* stop)
{
    *start = *stop = nullptr;
    if (!time_this(ctx, slot)) return;
    mlmc_ctx::Timed t;
    t.start = pool_event(ctx);
    t.stop = pool_event(ctx);
    if (!t.start || !t.stop) return;
    t.slot = slot;
    t.fine_steps = fine_steps;
    t.coarse_steps = coarse_steps;
    ctx->pending.push_back(t);
    *start = t.start;
    *stop = t.stop;
}

void timed_end(mlmc_ctx* ctx, int idx)
{
    if (idx < 0) return;
    hipEventRecord(ctx->pending[idx].stop, ctx->stream);
}

static void harvest_one(mlmc_ctx* ctx, const mlmc_ctx::Timed& t)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess) {
        mlmc_kernel_stat& s = ctx->stats[t.slot];
        s.launches += 1;
        s.ms += ms;
        s.fine_steps += t.fine_steps;
        s.coarse_steps += t.coarse_steps;
    }
    ctx->event_pool.push_back(t.start);
    ctx->event_pool.push_back(t.stop);
}

void harvest_timing(mlmc_ctx* ctx)
{
    for (auto& t : ctx->pending) harvest_one(ctx, t);
    ctx->pending.clear();
}

void harvest_ready(mlmc_ctx* ctx)
{
    // the events of one stream complete in order: stop at the first one
    // still outstanding
    size_t k = 0;
    while (k < ctx->pending.size() && hipEventQuery(ctx->pending[k].stop) == hipSuccess)
        harvest_one(ctx, ctx->pending[k++]);
    ctx->pending.erase(ctx->pending.begin(), ctx->pending.begin() + k);
}

// One launch over a range whose generator units share their counter word 2.
static mlmc_status enqueue_segment(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l,
                                   int M, uint64_t N, uint64_t seed, uint64_t offset, int precision,
                                   uint32_t stream, int coupled, LevelAcc* acc, double* d_pf,
                                   double* d_pc, const mlmc_cv* cv, bool spread, uint64_t n_call)
{
    const uint32_t mask = spread ? (uint32_t)(kSpread - 1) : 0u;
    const int dim = m.kind == MLMC_HESTON ? 2 : 1;
    if (cv) {
        if (precision != 32) return fail(ctx, MLMC_EINVAL, "the control variate runs in fp32 paths only");
        if (m.scheme != MLMC_EULER || m.antithetic)
            return fail(ctx, MLMC_EINVAL, "the control variate runs with plain Euler paths");
        if (p.kind == MLMC_DIGITAL_COND)
            return fail(ctx, MLMC_EINVAL, "the control variate takes the four plain payoffs");
        if (cv_in_dim(cv) != (m.kind == MLMC_HESTON ? 3 : 2))
            return fail(ctx, MLMC_EINVAL, "network inputs do not match the model (2: GBM, 3: Heston)");
        const double nf = (double)level_steps(l, M);
        auto a = make_args<float>(m, p, l, M, N, seed, offset, stream, coupled, acc, d_pf, d_pc);
        a.spread_mask = mask;
        set_counter_words(a, dim);
        // estimation may read the network from its table; training evaluates it
        const bool tab = cv_tabulated(cv) && stream != kStreamTrainNormal;
        hipError_t e;
        if (l == 0) {
            // one step from (0, S0): phi is the single value phi(0, S0)
            e = cv_ensure_phi0(cv, m, ctx->stream, tab);
            if (e != hipSuccess) return hip_fail(ctx, e, "phi(0, S0) launch");
            a.phi0 = cv_phi0_ptr(cv, tab);
            LaunchShape shape = choose_shape(ctx, m, p, l, M, 32, N);
            hipEvent_t t0, t1;
            timed_kernel(ctx, 0, (double)N, 0.0, &t0, &t1);
            e = launch_level(m, p, M, 32, &a, shape, ctx->stream, t0, t1);
        } else {
            // the tabulated sampler: GBM paths too few to fill the device run
            // on several lanes each (the plain sampler's rule on the call's
            // count), two samples per lane when there are lanes to spare
            int ppt = 1;
            if (tab) {
                a.split = split_lanes((int)nf, n_call ? n_call : N, ctx->num_cu, m.kind == MLMC_GBM);
                if (a.split == 1 && nf >= 4 && N >= (uint64_t)ctx->num_cu * 512) ppt = 2;
            }
            const uint64_t per_chunk = a.split > 1 ? 256 / a.split : 256 * (uint64_t)ppt;
            const uint64_t chunks = (N + per_chunk - 1) / per_chunk;
            // the tabulated sampler copies its level's table rows (<= 32 KiB)
            // into every block's LDS: four blocks per compute unit
            const uint64_t cap = (uint64_t)ctx->num_cu * (tab ? 4 : 8);
            const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>(chunks, cap));
            const int tix = timed_begin(ctx, l < 16 ? l : 15, (double)N * nf, (double)N * nf / M);
            e = cv_launch_level(cv, m, p, M, a, grid, ctx->stream, tab, ppt);
            timed_end(ctx, tix);
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "control-variate level launch");
        return MLMC_OK;
    }
    const LaunchShape shape = choose_shape(ctx, m, p, l, M, precision, N, n_call);
    const double nf = (double)level_steps(l, M);
    const double twins = (m.antithetic && l > 0) ? 2.0 : 1.0;   // fine paths per sample
    hipEvent_t t0, t1;
    timed_kernel(ctx, l < 16 ? l : 15, (double)N * nf * twins,
                 (coupled && l > 0) ? (double)N * nf / M : 0.0, &t0, &t1);
    const hipError_t e = launch_plain_segment(m, p, l, M, N, seed, offset, precision, stream, coupled,
                                              acc, d_pf, d_pc, spread, shape, ctx->stream, t0, t1);
    if (e != hipSuccess) return hip_fail(ctx, e, "level kernel launch");
    return MLMC_OK;
}

hipError_t launch_plain_segment(const mlmc_model& m, const mlmc_payoff& p, int l, int M, uint64_t N,
                                uint64_t seed, uint64_t offset, int precision, uint32_t stream,
                                int coupled, LevelAcc* acc, double* d_pf, double* d_pc, bool spread,
                                const LaunchShape& shape, hipStream_t st, hipEvent_t t0,
                                hipEvent_t t1)
{
    const uint32_t mask = spread ? (uint32_t)(kSpread - 1) : 0u;
    const int dim = m.kind == MLMC_HESTON ? 2 : 1;
    if (precision == 64) {
        auto a = make_args<double>(m, p, l, M, N, seed, offset, stream, coupled, acc, d_pf, d_pc);
        a.spread_mask = mask;
        set_counter_words(a, dim);
        return launch_level(m, p, M, 64, &a, shape, st, t0, t1);
    }
    auto a = make_args<float>(m, p, l, M, N, seed, offset, stream, coupled, acc, d_pf, d_pc);
    a.spread_mask = mask;
    a.split = (uint32_t)shape.split;
    set_counter_words(a, dim);
    return launch_level(m, p, M, 32, &a, shape, st, t0, t1);
}

mlmc_status enqueue_level(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l, int M,
                          uint64_t N, uint64_t seed, uint64_t offset, int precision, uint32_t stream,
                          int coupled, LevelAcc* acc, double* d_pf, double* d_pc, const mlmc_cv* cv,
                          bool spread)
{
    const uint64_t q = samples_per_unit(level_steps(l, M), m.kind == MLMC_HESTON ? 2 : 1);
    const uint64_t end = offset + N;
    for (uint64_t first = offset; first < end;) {
        const uint64_t stop = counter_segment_end(first, end, q);
        const uint64_t skip = first - offset;
        const mlmc_status st =
            enqueue_segment(ctx, m, p, l, M, stop - first, seed, first, precision, stream, coupled,
                            acc, d_pf ? d_pf + skip : nullptr, d_pc ? d_pc + skip : nullptr, cv,
                            spread, N);
        if (st) return st;
        first = stop;
    }
    return MLMC_OK;
}

static mlmc_status finish_level(mlmc_ctx* ctx, const mlmc_model& m, uint64_t N, int l, int M,
                                int coupled, mlmc_level_result* out)
{
    MLMC_HIP(ctx, hipMemcpyAsync(ctx->h_acc, ctx->d_acc, sizeof(LevelAcc) * kSpread,
                                 hipMemcpyDeviceToHost, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    harvest_timing(ctx);
    const LevelAcc r = fold_records(ctx->h_acc, kSpread);
    if (out) {
        out->sum_y = r.sum[0];
        out->sum_y2 = r.sum[1];
        out->sum_pf = r.sum[2];
        out->sum_pf2 = r.sum[3];
        out->sum_pc = r.sum[4];
        out->sum_pc2 = r.sum[5];
        out->cost = (double)N * (coupled ? level_cost(m, l, M) : std::pow((double)M, (double)l));
        out->n = N;
        out->n_nonfinite = r.n_nonfinite;
    }
    if (r.n_nonfinite)
        return fail(ctx, MLMC_ENONFINITE,
                    std::to_string(r.n_nonfinite) + " non-finite samples left out of the sums");
    return MLMC_OK;
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

mlmc_status mlmc_ctx_create(int device, mlmc_ctx** out)
{
    if (!out) return MLMC_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return MLMC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MLMC_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MLMC_EDEVICE;
    mlmc_ctx* ctx = new (std::nothrow) mlmc_ctx();
    if (!ctx) return MLMC_ENOMEM;
    ctx->device = device;
    ctx->num_cu = prop.multiProcessorCount;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_acc, sizeof(LevelAcc) * kAccSlots);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_acc, sizeof(LevelAcc) * kAccSlots);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_tmp, sizeof(double) * 4 * MLMC_MAX_LEVELS);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_tmp, sizeof(double) * 4 * MLMC_MAX_LEVELS);
    if (e != hipSuccess) {
        mlmc_ctx_destroy(ctx);
        return e == hipErrorOutOfMemory ? MLMC_ENOMEM : MLMC_EDEVICE;
    }
    ctx->stream = ctx->own_stream;
    *out = ctx;
    return MLMC_OK;
}

mlmc_status mlmc_ctx_destroy(mlmc_ctx* ctx)
{
    if (!ctx) return MLMC_OK;
    hipSetDevice(ctx->device);
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    free_driver(ctx);
    free_persistent(ctx);
    for (auto& t : ctx->pending) {
        hipEventDestroy(t.start);
        hipEventDestroy(t.stop);
    }
    for (auto e : ctx->event_pool) hipEventDestroy(e);
    if (ctx->d_acc) hipFree(ctx->d_acc);
    if (ctx->h_acc) hipHostFree(ctx->h_acc);
    if (ctx->d_tmp) hipFree(ctx->d_tmp);
    if (ctx->h_tmp) hipHostFree(ctx->h_tmp);
    if (ctx->own_stream) hipStreamDestroy(ctx->own_stream);
    delete ctx;
    return MLMC_OK;
}

mlmc_status mlmc_set_stream(mlmc_ctx* ctx, void* hip_stream)
{
    if (!ctx) return MLMC_EINVAL;
    // launches on the old stream must end before the new stream's start:
    // they share the context's buffers
    if (ctx->stream) MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->own_stream;
    return MLMC_OK;
}

const char* mlmc_last_error(const mlmc_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

mlmc_status mlmc_set_timing_mask(mlmc_ctx* ctx, uint32_t slot_mask)
{
    if (!ctx) return MLMC_EINVAL;
    if (slot_mask >> MLMC_STAT_SLOTS)
        return fail(ctx, MLMC_EINVAL, "slot mask has bits beyond the statistics slots");
    if (ctx->stream) MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    harvest_timing(ctx);
    ctx->timing = slot_mask;
    for (auto& n : ctx->timing_seen) n = 0;
    if (slot_mask)
        for (auto& s : ctx->stats) s = mlmc_kernel_stat{};
    return MLMC_OK;
}

mlmc_status mlmc_set_timing_stride(mlmc_ctx* ctx, uint32_t stride)
{
    if (!ctx) return MLMC_EINVAL;
    if (stride < 1) return fail(ctx, MLMC_EINVAL, "stride must be >= 1");
    ctx->timing_stride = stride;
    for (auto& n : ctx->timing_seen) n = 0;
    return MLMC_OK;
}

mlmc_status mlmc_set_timing_paused(mlmc_ctx* ctx, int paused)
{
    if (!ctx) return MLMC_EINVAL;
    ctx->timing_paused = paused != 0;
    return MLMC_OK;
}

mlmc_status mlmc_set_timing(mlmc_ctx* ctx, int on)
{
    return mlmc_set_timing_mask(ctx, on ? (1u << MLMC_STAT_SLOTS) - 1u : 0u);
}

mlmc_status mlmc_kernel_stats(mlmc_ctx* ctx, mlmc_kernel_stat* out)
{
    if (!ctx || !out) return MLMC_EINVAL;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    harvest_timing(ctx);
    for (int i = 0; i < MLMC_STAT_SLOTS; ++i) out[i] = ctx->stats[i];
    return MLMC_OK;
}

mlmc_status mlmc_set_launch(mlmc_ctx* ctx, int block, int ppt)
{
    if (!ctx) return MLMC_EINVAL;
    if (block == 0) {
        ctx->launch_block = ctx->launch_ppt = 0;
        return MLMC_OK;
    }
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024)
        return fail(ctx, MLMC_EINVAL, "block must be 64, 128, 256, 512 or 1024");
    if (ppt != 1 && ppt != 2 && ppt != 4) return fail(ctx, MLMC_EINVAL, "ppt must be 1, 2 or 4");
    ctx->launch_block = block;
    ctx->launch_ppt = ppt;
    return MLMC_OK;
}

static mlmc_status level_common(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                                int l, int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                                int precision, const mlmc_cv* cv, double* d_pf, double* d_pc,
                                uint32_t stream, int coupled, mlmc_level_result* out)
{
    mlmc_status st = check_level_args(ctx, model, payoff, l, M, precision);
    if (st) return st;
    if (cv && precision != 32)
        return fail(ctx, MLMC_EINVAL, "the control variate runs in fp32 paths only");
    if (!coupled && model->antithetic)
        return fail(ctx, MLMC_EINVAL, "the antithetic twin belongs to level differences");
    if (N > (1ull << 40)) return fail(ctx, MLMC_EINVAL, "N too large (max 2^40 per call)");
    if ((path_offset + N) >> 56) return fail(ctx, MLMC_EINVAL, "path index beyond 2^56");
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, zero_records(ctx->d_acc, kSpread, ctx->stream));
    st = enqueue_level(ctx, *model, *payoff, l, M, N, seed, path_offset, precision, stream, coupled,
                       ctx->d_acc, d_pf, d_pc, cv, true);
    if (st) return st;
    return finish_level(ctx, *model, N, l, M, coupled, out);
}

mlmc_status mlmc_level(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff, int l,
                       int M, uint64_t N, uint64_t seed, uint64_t path_offset, int precision,
                       const mlmc_cv* cv, mlmc_level_result* out)
{
    if (!out) return fail(ctx, MLMC_EINVAL, "out must not be NULL");
    return level_common(ctx, model, payoff, l, M, N, seed, path_offset, precision, cv, nullptr,
                        nullptr, kStreamNormal, 1, out);
}

mlmc_status mlmc_level_paths(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                             int l, int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                             int precision, const mlmc_cv* cv, double* d_pf, double* d_pc,
                             mlmc_level_result* out)
{
    if (N && (!d_pf || !d_pc)) return fail(ctx, MLMC_EINVAL, "d_pf and d_pc must be device arrays");
    return level_common(ctx, model, payoff, l, M, N, seed, path_offset, precision, cv, d_pf, d_pc,
                        kStreamNormal, 1, out);
}

mlmc_status mlmc_stdmc(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff, int L,
                       int M, uint64_t N, uint64_t seed, uint64_t path_offset, int precision,
                       mlmc_level_result* out)
{
    if (!out) return fail(ctx, MLMC_EINVAL, "out must not be NULL");
    return level_common(ctx, model, payoff, L, M, N, seed, path_offset, precision, nullptr, nullptr,
                        nullptr, kStreamStdMC, 0, out);
}

mlmc_status mlmc_philox_words(mlmc_ctx* ctx, uint64_t seed, int level, uint64_t s0, uint32_t stream,
                              uint32_t nblocks, uint64_t npaths, uint32_t* d_out)
{
    if (!ctx) return MLMC_EINVAL;
    if (!d_out && npaths && nblocks) return fail(ctx, MLMC_EINVAL, "d_out must not be NULL");
    if (level < 0 || level > 255) return fail(ctx, MLMC_EINVAL, "level must be in 0..255");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, launch_philox_words(seed, level, s0, stream, nblocks, npaths, d_out, ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return MLMC_OK;
}

mlmc_status mlmc_normals(mlmc_ctx* ctx, uint64_t seed, int level, uint64_t s0, uint32_t stream,
                         int dim, int nsteps, uint64_t npaths, int precision, double* d_out)
{
    if (!ctx) return MLMC_EINVAL;
    if ((dim != 1 && dim != 2) || nsteps < 0 || (precision != 32 && precision != 64))
        return fail(ctx, MLMC_EINVAL, "dim must be 1 or 2, precision 32 or 64");
    if (!d_out && npaths && nsteps) return fail(ctx, MLMC_EINVAL, "d_out must not be NULL");
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    MLMC_HIP(ctx, launch_normals(seed, level, s0, stream, dim, nsteps, npaths, precision, d_out,
                                 ctx->stream));
    MLMC_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return MLMC_OK;
}

}  // extern "C"
