// mlmc_level_noalloc: the level estimator sums of mlmc_level with no context
// and no device allocation, for callers that cannot allocate (code under HIP
// graph capture, tight serving loops).
//
// The only scratch the level kernels need is one spread group of level
// records (partial sums that the blocks add into, block b into record
// b mod kSpread).  Here that group is a file-scope device array; each device
// holds its own copy for the life of the process.  Host code never passes the
// array's name to a kernel: on a device's first call its address is taken
// with hipGetSymbolAddress (with that device current) and kept per device.
// Every call on a device uses that one array: a fill kernel clears it, the
// level kernels add into it, and a one-thread kernel folds it into the
// caller's device result, all on the caller's stream.  Calls that overlap on
// one device (other streams, other host threads) race on the array.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "context.hpp"

namespace mlmc {

// One spread group: kSpread records of 64 bytes (4 KiB) per device.
constexpr int kScratchRecords = kSpread;
static __device__ __align__(256) LevelAcc scratch[kScratchRecords];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::atomic<int> ready{0};   // 1: ptr and num_cu are set
    LevelAcc* ptr = nullptr;     // this device's copy of `scratch`
    int num_cu = 0;
};

DeviceScratch g_dev[kMaxDevices];
std::mutex g_setup;

void put_err(char* err, size_t len, const char* msg)
{
    if (err && len) {
        std::strncpy(err, msg, len - 1);
        err[len - 1] = '\0';
    }
}

// Address of the scratch array on the current device `dev`, set up once.
hipError_t scratch_for(int dev, DeviceScratch** out)
{
    DeviceScratch& d = g_dev[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(g_setup);
        if (!d.ready.load(std::memory_order_relaxed)) {
            void* p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            int cu = 0;
            e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            d.ptr = static_cast<LevelAcc*>(p);
            d.num_cu = cu;
            d.ready.store(1, std::memory_order_release);
        }
    }
    *out = &d;
    return hipSuccess;
}

}  // namespace

// Sum of the group in record order (the order mlmc_level folds in), written
// as the caller's result.
__global__ void fold_to_result_kernel(const LevelAcc* group, mlmc_level_result* out, uint64_t N,
                                      double cost)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const LevelAcc r = fold_records(group, kScratchRecords);
    out->sum_y = r.sum[0];
    out->sum_y2 = r.sum[1];
    out->sum_pf = r.sum[2];
    out->sum_pf2 = r.sum[3];
    out->sum_pc = r.sum[4];
    out->sum_pc2 = r.sum[5];
    out->cost = cost;
    out->n = N;
    out->n_nonfinite = r.n_nonfinite;
}

}  // namespace mlmc

using namespace mlmc;

extern "C" mlmc_status mlmc_level_noalloc(const mlmc_model* model, const mlmc_payoff* payoff, int l,
                                          int M, uint64_t N, uint64_t seed, uint64_t path_offset,
                                          int precision, void* hip_stream,
                                          mlmc_level_result* d_out, char* err, size_t err_len)
{
    put_err(err, err_len, "");
    if (const char* why = level_args_error(model, payoff, l, M, precision)) {
        put_err(err, err_len, why);
        return MLMC_EINVAL;
    }
    if (!d_out) {
        put_err(err, err_len, "d_out must be a device pointer to one mlmc_level_result");
        return MLMC_EINVAL;
    }
    // the group's size does not grow with N: any count the sampler accepts fits
    if (N > (1ull << 40)) {
        put_err(err, err_len, "N too large (max 2^40 per call)");
        return MLMC_EINVAL;
    }
    if ((path_offset + N) >> 56) {
        put_err(err, err_len, "path index beyond 2^56");
        return MLMC_EINVAL;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        put_err(err, err_len, "no usable current HIP device");
        return MLMC_EDEVICE;
    }
    DeviceScratch* ds = nullptr;
    e = scratch_for(dev, &ds);
    if (e != hipSuccess) {
        put_err(err, err_len, hipGetErrorString(e));
        return MLMC_EDEVICE;
    }
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    LevelAcc* group = ds->ptr;
    e = zero_records(group, kScratchRecords, st);
    const mlmc_model& m = *model;
    const mlmc_payoff& p = *payoff;
    int nf = 1;
    for (int i = 0; i < l; ++i) nf *= M;
    const uint64_t q = samples_per_unit(nf, m.kind == MLMC_HESTON ? 2 : 1);
    // one launch per run of generator units that share counter word 2
    for (uint64_t first = path_offset, end = path_offset + N; e == hipSuccess && first < end;) {
        const uint64_t stop = counter_segment_end(first, end, q);
        const LaunchShape shape =
            default_shape(m, p, l, M, precision, stop - first, N, ds->num_cu, 0, 0, 0, 0);
        e = launch_plain_segment(m, p, l, M, stop - first, seed, first, precision, kStreamNormal, 1,
                                 group, nullptr, nullptr, true, shape, st);
        first = stop;
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fold_to_result_kernel, dim3(1), dim3(64), 0, st, group, d_out, N,
                           (double)N * level_cost(m, l, M));
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        put_err(err, err_len, hipGetErrorString(e));
        return MLMC_EDEVICE;
    }
    return MLMC_OK;
}
