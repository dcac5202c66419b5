// Internal definitions shared by the runtime and the workload launchers.
#pragma once
#include <hip/hip_runtime.h>

#include "hr.h"
#include "hr_device.h"

static_assert(sizeof(hr_race) == sizeof(hr_race_rec), "hr_race layout");

struct hr_region {
    const void* data;
    size_t elems;        // 4-byte elements
    uint64_t* shadow;    // one 8-byte word per element
};

struct hr_ctx_s {
    hipStream_t stream;
    int device;
    hr_config cfg;
    hr_region reg[HR_MAX_REGIONS];
    uint32_t n_reg;
    hr_race_rec* ring;
    uint32_t* ctr;
    unsigned long long* count;   // HR_COUNT_SLOTS debug counters
    uint32_t launch_seq;     // launches since the job started
    uint64_t shadow_bytes;
};

hipStream_t hr_stream(hr_ctx c, void* stream);
void hr_fill_args(hr_ctx c, hr_kargs* a);

#define HR_HIP_CHECK(expr)                              \
    do {                                                \
        if ((expr) != hipSuccess) return HR_E_HIP;      \
    } while (0)

// Launch a kernel and return HR_E_HIP if the launch itself failed.  The HIP
// runtime is shared with the caller (PyTorch), and hipGetLastError also
// returns errors left behind by unrelated earlier calls of this thread, so
// the stale value is cleared before the launch.
#define HR_LAUNCH(...)                                          \
    do {                                                        \
        (void)hipGetLastError();                                \
        hipLaunchKernelGGL(__VA_ARGS__);                        \
        if (hipGetLastError() != hipSuccess) return HR_E_HIP;   \
    } while (0)
