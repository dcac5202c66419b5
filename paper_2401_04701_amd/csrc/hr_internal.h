// Internal definitions shared by the runtime, the workload launchers and the
// batch executor.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hr.h"
#include "hr_device.h"

static_assert(sizeof(hr_race) == sizeof(hr_race_rec), "hr_race layout");

// One device allocation of shadow words (a region's own, or a batch arena).
struct hr_alloc {
    uint64_t* mem;
    size_t words;
    bool live;
};

struct hr_region {
    const void* data;    // monitored buffer
    size_t elems;        // 4-byte elements
    uint64_t* shadow;    // one 8-byte word per element, inside allocs[alloc]
    uint32_t alloc;
    bool live;
    bool monitored;      // cleared by hr_region_enable(..., 0)
};

struct hr_ctx_s {
    hipStream_t stream;
    int device;
    hr_config cfg;
    std::vector<hr_alloc> allocs;
    std::vector<hr_region> reg;      // region ids index this vector; never reused
    hr_race_rec* ring;
    uint32_t* ctr;
    unsigned long long* count;       // HR_COUNT_SLOTS debug counters
    uint32_t launch_seq;             // launches since the job started
    uint64_t shadow_bytes;           // live shadow memory
    std::vector<hr_race> carried;    // global races recovered before a shadow clear
};

hipStream_t hr_stream(hr_ctx c, void* stream);
hr_env hr_make_env(hr_ctx c);
void hr_fill_args(hr_ctx c, hr_kargs* a);
// A region usable through kernel arguments (id < HR_MAX_REGIONS), registered
// for `data` and holding at least min_elems elements.
bool hr_region_ok(hr_ctx c, uint32_t r, const void* data, size_t min_elems);
// Allocate `words` cleared shadow words as a new allocation.
hr_status hr_new_alloc(hr_ctx c, size_t words, uint32_t* alloc_out);
uint32_t hr_new_region(hr_ctx c, const void* data, size_t elems, uint64_t* shadow, uint32_t alloc);
void hr_free_alloc(hr_ctx c, uint32_t alloc);
hipError_t hr_fill64(uint64_t* p, size_t n, hipStream_t s);
hipError_t hr_fill32(uint32_t* p, size_t n, hipStream_t s);

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
