// Device microbenchmarks that give the roofline denominators of the checker:
// streaming copy (HBM bandwidth, also the calibration kernel for the HBM
// byte counters), agent-scope 64-bit compare-and-swap and exchange on
// distinct words (coalesced, scattered in 64 KiB windows, or spread over the
// whole array), agent-scope 64-bit atomic loads, and 32-bit LDS
// compare-and-swap (alone, and after a load as the LDS hook does it).
#include <hip/hip_runtime.h>

#include "hr.h"
#include "hr_internal.h"

namespace {

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src,
                                              uint4* __restrict__ dst, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// Word w holds `round` before round `round`; every compare-and-swap succeeds.
// scatter 1 permutes word indices inside each 64 KiB window so that the
// lanes of a wave touch different cache lines; scatter 2 (n a power of two)
// spreads consecutive indices over the whole array.
__device__ __forceinline__ size_t peak_index(size_t i, size_t n, uint32_t scatter)
{
    if (!scatter) return i;
    if (scatter == 2 && (n & (n - 1)) == 0)
        return (i * 0x9E3779B1ull) & (n - 1);       // odd multiplier: a bijection mod n
    const size_t win = 8192;                        // 64 KiB of 8-byte words
    const size_t base = i & ~(win - 1);
    const size_t j = ((i & (win - 1)) * 4099u) & (win - 1);   // odd multiplier: a bijection
    const size_t k = base + j;
    return k < n ? k : i;
}

// op 0: compare-and-swap round -> round+1; op 1: exchange in round+1 and
// check the returned value.  Either way a failure means the word did not
// hold `round`.
template <int OP>
__global__ __launch_bounds__(256) void k_atomic(uint64_t* __restrict__ w, size_t n, uint32_t round,
                                                uint32_t scatter, uint32_t* __restrict__ fails)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (; i < n; i += stride) {
        uint64_t* p = w + peak_index(i, n, scatter);
        if (OP == 0) {
            uint64_t expect = round;
            if (!__hip_atomic_compare_exchange_strong(p, &expect, (uint64_t)round + 1,
                                                      __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT))
                ++bad;
        } else {
            if (__hip_atomic_exchange(p, (uint64_t)round + 1, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT) != round)
                ++bad;
        }
    }
    if (bad) atomicAdd(fails, bad);
}

__global__ __launch_bounds__(256) void k_load(const uint64_t* __restrict__ w, size_t n,
                                              uint32_t scatter, uint64_t* __restrict__ sink)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (; i < n; i += stride)
        acc ^= __hip_atomic_load(w + peak_index(i, n, scatter), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
    if (acc == 0x9E3779B97F4A7C15ull) *sink = acc;    // keeps the loads alive
}

// LDS 32-bit compare-and-swap: every thread owns word threadIdx.x of a
// block-local array and takes it from r to r+1 for r = 0 .. iters-1
// (op 0), or first loads it and swaps from the loaded value (op 1, the LDS
// hook's load + compare-and-swap).  Lanes of a wave hit distinct banks.
template <int OP>
__global__ __launch_bounds__(1024) void k_lds_cas(uint32_t iters, uint32_t* __restrict__ fails)
{
    __shared__ uint32_t w[1024];
    uint32_t* p = w + threadIdx.x;
    *p = 0;
    uint32_t bad = 0;
    for (uint32_t r = 0; r < iters; ++r) {
        uint32_t expect = OP == 0 ? r
                                  : __hip_atomic_load(p, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
        if (!__hip_atomic_compare_exchange_strong(p, &expect, expect + 1, __ATOMIC_RELAXED,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            ++bad;
    }
    if (*p != iters) ++bad;
    if (bad) atomicAdd(fails, bad);
}

unsigned grid_for(size_t n)
{
    const size_t blocks = (n + 255) / 256;
    return (unsigned)(blocks < 65536 ? blocks : 65536);
}

}  // namespace

extern "C" hr_status hr_peak_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream)
{
    if (!src_dev || !dst_dev || bytes % 16) return HR_E_INVAL;
    const size_t n = bytes / 16;
    if (n == 0) return HR_OK;
    HR_LAUNCH(k_copy, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (const uint4*)src_dev,
              (uint4*)dst_dev, n);
    return HR_OK;
}

extern "C" hr_status hr_peak_atomic(uint64_t* words_dev, size_t n, uint32_t op, uint32_t round,
                                    uint32_t scatter, uint32_t* fails_dev, uint32_t blocks,
                                    void* stream)
{
    if (!words_dev || !fails_dev || n == 0 || op > 1 || blocks > 65536) return HR_E_INVAL;
    const unsigned grid = blocks ? blocks : grid_for(n);
    if (op == 0)
        HR_LAUNCH(k_atomic<0>, dim3(grid), dim3(256), 0, (hipStream_t)stream, words_dev, n, round,
                  scatter, fails_dev);
    else
        HR_LAUNCH(k_atomic<1>, dim3(grid), dim3(256), 0, (hipStream_t)stream, words_dev, n, round,
                  scatter, fails_dev);
    return HR_OK;
}

extern "C" hr_status hr_peak_load(const uint64_t* words_dev, size_t n, uint32_t scatter,
                                  uint64_t* sink_dev, void* stream)
{
    if (!words_dev || !sink_dev || n == 0) return HR_E_INVAL;
    HR_LAUNCH(k_load, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, words_dev, n, scatter,
              sink_dev);
    return HR_OK;
}

extern "C" hr_status hr_peak_lds(uint32_t blocks, uint32_t iters, uint32_t op, uint32_t* fails_dev,
                                 void* stream)
{
    if (!fails_dev || blocks == 0 || iters == 0 || op > 1) return HR_E_INVAL;
    if (op == 0)
        HR_LAUNCH(k_lds_cas<0>, dim3(blocks), dim3(1024), 0, (hipStream_t)stream, iters, fails_dev);
    else
        HR_LAUNCH(k_lds_cas<1>, dim3(blocks), dim3(1024), 0, (hipStream_t)stream, iters, fails_dev);
    return HR_OK;
}
