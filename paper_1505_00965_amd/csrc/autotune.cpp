// Launch-shape autotuner: picks block size and samples per lane for the
// level sampler (per model, payoff, precision, M and level class) and block
// size, samples per lane and resident blocks per compute unit for the
// persistent kernel, by timing candidates with HIP events on the device
// itself.  Results are results of measurement, so they are cached in a small
// JSON file keyed by GPU architecture, compute-unit count and HIP runtime
// version; a later context on the same machine reads them back instead of
// measuring again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "context.hpp"

namespace mlmc {

// Level classes: levels 0..5 each (an adaptive run's launch sizes differ by
// level: N_l falls about as fast as the fine steps M^l grow, so each level's
// launches have a size of their own) and the deeper levels together.
constexpr int kTuneClasses = 7;
int level_class(int l, int M)
{
    (void)M;
    return l < kTuneClasses - 1 ? l : kTuneClasses - 1;
}

// The scheme and the antithetic twin change the kernel (register use, work
// per step), so they are part of the key.
static std::string tune_key(const mlmc_model& m, int payoff, int precision, int M, int cls)
{
    char b[80];
    std::snprintf(b, sizeof b, "level:%d:%d:%d:%d:%d:%d:%d", m.kind, m.scheme, m.antithetic, payoff,
                  precision, M, cls);
    return b;
}

static std::string machine_key(const mlmc_ctx* ctx)
{
    hipDeviceProp_t prop;
    hipGetDeviceProperties(&prop, ctx->device);
    int rt = 0;
    hipRuntimeGetVersion(&rt);
    char b[160];
    std::snprintf(b, sizeof b, "%s|cu%d|hip%d", prop.gcnArchName, prop.multiProcessorCount, rt);
    return b;
}

// Minimal JSON of the form {"machine": {"key": [a, b, c], ...}, ...}.
static std::map<std::string, std::map<std::string, std::vector<int>>> read_cache(const std::string& path)
{
    std::map<std::string, std::map<std::string, std::vector<int>>> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    auto skip = [&]() { while (i < s.size() && std::strchr(" \t\r\n,:", s[i])) ++i; };
    auto str = [&](std::string& v) -> bool {
        skip();
        if (i >= s.size() || s[i] != '"') return false;
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) return false;
        v = s.substr(i + 1, j - i - 1);
        i = j + 1;
        return true;
    };
    skip();
    if (i >= s.size() || s[i] != '{') return out;
    ++i;
    for (;;) {
        std::string mk;
        if (!str(mk)) break;
        skip();
        if (i >= s.size() || s[i] != '{') break;
        ++i;
        for (;;) {
            std::string k;
            if (!str(k)) break;
            skip();
            if (i >= s.size() || s[i] != '[') break;
            ++i;
            std::vector<int> v;
            for (;;) {
                skip();
                if (i < s.size() && s[i] == ']') { ++i; break; }
                char* end = nullptr;
                const long x = std::strtol(s.c_str() + i, &end, 10);
                if (end == s.c_str() + i) return out;
                v.push_back((int)x);
                i = end - s.c_str();
            }
            out[mk][k] = v;
        }
        skip();
        if (i < s.size() && s[i] == '}') ++i;
    }
    return out;
}

static bool write_cache(const std::string& path,
                        const std::map<std::string, std::map<std::string, std::vector<int>>>& c)
{
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t a = 0;
    for (const auto& m : c) {
        std::fprintf(f, "  \"%s\": {\n", m.first.c_str());
        size_t b = 0;
        for (const auto& e : m.second) {
            std::fprintf(f, "    \"%s\": [", e.first.c_str());
            for (size_t k = 0; k < e.second.size(); ++k)
                std::fprintf(f, "%s%d", k ? ", " : "", e.second[k]);
            std::fprintf(f, "]%s\n", ++b < m.second.size() ? "," : "");
        }
        std::fprintf(f, "  }%s\n", ++a < c.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool tuned_shape(const mlmc_ctx* ctx, const mlmc_model& m, int payoff, int precision, int M, int l,
                 int* block, int* ppt)
{
    if (ctx->tuned.empty()) return false;   // every launch asks: skip the key when nothing is tuned
    auto it = ctx->tuned.find(tune_key(m, payoff, precision, M, level_class(l, M)));
    if (it == ctx->tuned.end() || it->second.size() < 2) return false;
    *block = it->second[0];
    *ppt = it->second[1];
    return true;
}

// Time one level launch shape (median of 5 after a warm-up), milliseconds.
static float time_shape(mlmc_ctx* ctx, const mlmc_model& m, const mlmc_payoff& p, int l, int M,
                        uint64_t N, int precision, int block, int ppt, mlmc_status* st)
{
    const int saved_b = ctx->launch_block, saved_p = ctx->launch_ppt;
    ctx->launch_block = block;
    ctx->launch_ppt = ppt;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    float best[5] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
    for (int rep = 0; rep < 6 && !*st; ++rep) {
        hipEventRecord(a, ctx->stream);
        *st = enqueue_level(ctx, m, p, l, M, N, 12345, 0, precision, kStreamNormal, 1, ctx->d_acc,
                            nullptr, nullptr, nullptr, true);
        hipEventRecord(b, ctx->stream);
        if (hipEventSynchronize(b) != hipSuccess) *st = MLMC_EDEVICE;
        float ms = 0.f;
        hipEventElapsedTime(&ms, a, b);
        if (rep > 0) best[rep - 1] = ms;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    ctx->launch_block = saved_b;
    ctx->launch_ppt = saved_p;
    std::sort(best, best + 5);
    return best[2];
}

}  // namespace mlmc

using namespace mlmc;

extern "C" {

mlmc_status mlmc_autotune(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff, int M,
                          int precision, const char* cache_path)
{
    if (!ctx) return MLMC_EINVAL;
    mlmc_status st = check_level_args(ctx, model, payoff, 0, M, precision);
    if (st) return st;
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    std::string path;
    if (cache_path && *cache_path) path = cache_path;
    else if (const char* e = std::getenv("MLMC_TUNE_CACHE")) path = e;
    const std::string mk = machine_key(ctx);
    auto cache = path.empty() ? decltype(read_cache(path)){} : read_cache(path);
    bool dirty = false;
    const int blocks[] = {64, 128, 256, 512, 1024};
    const int ppts32[] = {1, 2, 4};
    // each class at its first level, on 2^25 fine path steps per launch:
    // N_l M^l is about level-independent in an adaptive run, and 2^25 is its
    // size near RMSE 2e-5 S0 (smaller launches are cut down further by the
    // fill rule of the default shape)
    for (int cls = 0; cls < kTuneClasses; ++cls) {
        const std::string key = tune_key(*model, payoff->kind, precision, M, cls);
        auto mit = cache.find(mk);
        if (mit != cache.end() && mit->second.count(key)) {
            ctx->tuned[key] = mit->second[key];
            continue;
        }
        const int l = cls;
        double nf = 1.0;
        for (int i = 0; i < l; ++i) nf *= M;
        const uint64_t N = (uint64_t)std::max(1.0, (double)(1ull << 25) / nf);
        float best = 1e30f;
        int bb = 256, bp = precision == 64 ? 1 : 2;
        for (int b : blocks)
            for (int p : ppts32) {
                if (precision == 64 && p != 1) continue;
                if (cls == 0 && p == 4) continue;
                const float ms = time_shape(ctx, *model, *payoff, l, M, N, precision, b, p, &st);
                if (st) return st;
                if (ms < best) { best = ms; bb = b; bp = p; }
            }
        ctx->tuned[key] = {bb, bp};
        cache[mk][key] = {bb, bp};
        dirty = true;
    }
    if (dirty && !path.empty() && !write_cache(path, cache))
        return fail(ctx, MLMC_EINVAL, "could not write the tuning cache " + path);
    return MLMC_OK;
}

mlmc_status mlmc_autotune_persistent(mlmc_ctx* ctx, const mlmc_model* model,
                                     const mlmc_payoff* payoffs, int npayoffs, int M, int L,
                                     const char* cache_path, int* shape)
{
    if (!ctx) return MLMC_EINVAL;
    if (!model || !payoffs) return fail(ctx, MLMC_EINVAL, "model and payoffs must not be NULL");
    if (npayoffs < 1 || npayoffs > 4) return fail(ctx, MLMC_EINVAL, "npayoffs must be in 1..4");
    if (L < 0 || L > 15) return fail(ctx, MLMC_EINVAL, "L must be in 0..15");
    for (int k = 0; k < npayoffs; ++k) {
        const mlmc_status st = check_level_args(ctx, model, &payoffs[k], L, M, 32);
        if (st) return st;
    }
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    std::string path;
    if (cache_path && *cache_path) path = cache_path;
    else if (const char* e = std::getenv("MLMC_TUNE_CACHE")) path = e;
    const std::string mk = machine_key(ctx);
    auto cache = path.empty() ? decltype(read_cache(path)){} : read_cache(path);
    // every payoff of the batch is part of the key: the mix sets the work
    char kb[96];
    std::snprintf(kb, sizeof kb, "persist:%d:%d:%d:%d:%d:", model->kind, model->scheme, M, L,
                  npayoffs);
    std::string key = kb;
    for (int k = 0; k < npayoffs; ++k) key += std::to_string(payoffs[k].kind) + (k + 1 < npayoffs ? "," : "");
    auto mit = cache.find(mk);
    if (mit != cache.end() && mit->second.count(key) && mit->second[key].size() == 3) {
        const auto& v = mit->second[key];
        if (shape) std::memcpy(shape, v.data(), 3 * sizeof(int));
        return mlmc_set_persistent_launch(ctx, v[0], v[1], v[2]);
    }
    // the caller's levels and payoffs at an MLMC-shaped count, N_l = 2^24 M^-l
    std::vector<uint64_t> N((size_t)npayoffs * (L + 1));
    for (int k = 0; k < npayoffs; ++k) {
        double n = (double)(1ull << 24);
        for (int l = 0; l <= L; ++l, n /= M) N[(size_t)k * (L + 1) + l] = (uint64_t)std::max(1.0, n);
    }
    std::vector<mlmc_level_result> out((size_t)npayoffs * (L + 1));
    const int blocks[] = {128, 256, 512};
    const int bpcs[] = {2, 4, 8};
    const int ppts[] = {1, 2, 4};
    double best = 1e30;
    int bb = 256, bp = 1, bc = 4;
    for (int b : blocks)
        for (int c : bpcs) {
            if (b * c > 2048) continue;   // resident: at most 2048 threads per compute unit
            for (int p : ppts) {
                mlmc_status st = mlmc_set_persistent_launch(ctx, b, p, c);
                double t[3] = {0, 0, 0};
                // the first call captures the graph; then the median of three
                for (int rep = 0; rep < 4 && !st; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    st = mlmc_levels_batch(ctx, model, payoffs, npayoffs, M, L, N.data(), nullptr,
                                           12345, out.data());
                    if (st == MLMC_ENONFINITE) st = MLMC_OK;   // timed all the same
                    const auto t1 = std::chrono::steady_clock::now();
                    if (rep > 0) t[rep - 1] = std::chrono::duration<double>(t1 - t0).count();
                }
                if (st) {
                    mlmc_set_persistent_launch(ctx, 0, 0, 0);
                    return st;
                }
                std::sort(t, t + 3);
                if (t[1] < best) { best = t[1]; bb = b; bp = p; bc = c; }
            }
        }
    cache[mk][key] = {bb, bp, bc};
    const mlmc_status st = mlmc_set_persistent_launch(ctx, bb, bp, bc);
    if (st) return st;
    if (shape) {
        shape[0] = bb;
        shape[1] = bp;
        shape[2] = bc;
    }
    if (!path.empty() && !write_cache(path, cache))
        return fail(ctx, MLMC_EINVAL, "could not write the tuning cache " + path);
    return MLMC_OK;
}

mlmc_status mlmc_autotune_run(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                              const mlmc_run_opts* opts, const char* cache_path, int* shape)
{
    if (!ctx) return MLMC_EINVAL;
    if (!model || !payoff || !opts) return fail(ctx, MLMC_EINVAL, "model, payoff and opts must not be NULL");
    if (opts->persistent != 1)
        return fail(ctx, MLMC_EINVAL, "the run autotuner tunes the device-planned form (persistent = 1)");
    mlmc_status st = check_level_args(ctx, model, payoff, 0, opts->M, opts->precision);
    if (st) return st;
    ctx->err.clear();
    MLMC_HIP(ctx, hipSetDevice(ctx->device));
    std::string path;
    if (cache_path && *cache_path) path = cache_path;
    else if (const char* e = std::getenv("MLMC_TUNE_CACHE")) path = e;
    const std::string mk = machine_key(ctx);
    auto cache = path.empty() ? decltype(read_cache(path)){} : read_cache(path);
    // the run's whole configuration is the key: it sets the batches
    char kb[192];
    std::snprintf(kb, sizeof kb, "run:%d:%d:%d:%d:%.9g:%d:%d:%d:%llu:%.9g:%.9g", model->kind,
                  model->scheme, payoff->kind, opts->M, opts->eps, opts->L_min, opts->L_max,
                  opts->precision, (unsigned long long)opts->n_pilot, opts->alpha, opts->beta);
    const std::string key = kb;
    auto mit = cache.find(mk);
    if (mit != cache.end() && mit->second.count(key) && mit->second[key].size() == 3) {
        const auto& v = mit->second[key];
        if (shape) std::memcpy(shape, v.data(), 3 * sizeof(int));
        return mlmc_set_persistent_launch(ctx, v[0], v[1], v[2]);
    }
    const int blocks[] = {128, 256, 512};
    const int bpcs[] = {2, 4, 8};
    const int ppts[] = {1, 2, 4};
    double best = 1e30;
    int bb = 256, bp = 1, bc = 4;
    mlmc_run_result res;
    for (int b : blocks)
        for (int c : bpcs) {
            if (b * c > 2048) continue;   // resident: at most 2048 threads per compute unit
            for (int p : ppts) {
                st = mlmc_set_persistent_launch(ctx, b, p, c);
                double t[3] = {0, 0, 0};
                // a warm-up run, then the median of three (the same seed: the
                // same batches for every shape)
                for (int rep = 0; rep < 4 && !st; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    st = mlmc_run(ctx, model, payoff, opts, &res);
                    if (st == MLMC_ENOTCONV) st = MLMC_OK;   // timed all the same
                    const auto t1 = std::chrono::steady_clock::now();
                    if (rep > 0) t[rep - 1] = std::chrono::duration<double>(t1 - t0).count();
                }
                if (st) {
                    mlmc_set_persistent_launch(ctx, 0, 0, 0);
                    return st;
                }
                std::sort(t, t + 3);
                if (t[1] < best) { best = t[1]; bb = b; bp = p; bc = c; }
            }
        }
    cache[mk][key] = {bb, bp, bc};
    st = mlmc_set_persistent_launch(ctx, bb, bp, bc);
    if (st) return st;
    if (shape) {
        shape[0] = bb;
        shape[1] = bp;
        shape[2] = bc;
    }
    if (!path.empty() && !write_cache(path, cache))
        return fail(ctx, MLMC_EINVAL, "could not write the tuning cache " + path);
    return MLMC_OK;
}

mlmc_status mlmc_tuned_shape(mlmc_ctx* ctx, const mlmc_model* model, const mlmc_payoff* payoff,
                             int l, int M, int precision, int* block, int* ppt)
{
    if (!ctx || !model || !payoff || !block || !ppt) return MLMC_EINVAL;
    if (!tuned_shape(ctx, *model, payoff->kind, precision, M, l, block, ppt)) {
        *block = 0;
        *ppt = 0;
    }
    return MLMC_OK;
}

}  // extern "C"
