// Internal definitions shared by the runtime, the workload launchers and the
// batch executor.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hr.h"
#include "hr_device.h"

static_assert(sizeof(hr_race) == sizeof(hr_race_rec), "hr_race layout");
static_assert(sizeof(hr_access_rec) == 32, "hr_access_rec layout");

// One device allocation of shadow words (a region's own, or a batch arena).
struct hr_alloc {
    uint64_t* mem;
    size_t words;
    bool live;
};

struct hr_region {
    const void* data;    // monitored buffer
    size_t elems;        // 4-byte elements
    uint64_t* shadow;    // its shadow words (8- or 4-byte), inside allocs[alloc]
    uint32_t alloc;
    bool live;
    bool monitored;      // cleared by hr_region_enable(..., 0)
    hr_lay lay = {};     // address-to-shadow map (zero: row-major, 1-D)
    uint32_t rows = 0;   // rows of a tiled map
};


struct hr_ctx_s {
    hipStream_t stream;
    int device;
    hr_config cfg;
    std::vector<hr_alloc> allocs;
    std::vector<hr_region> reg;      // region ids index this vector; never reused
    uint32_t* ctr;                   // counters, then (at HR_CTR_BYTES) the ring:
    hr_race_rec* ring;               // one allocation, so one copy reads both
    uint32_t last_head = 0;          // records the last report read
    unsigned long long* count;       // HR_COUNT_SLOTS debug counters
    hr_access_rec* log;              // access log (HR_CFG_ACCESS_LOG), or null
    uint16_t* fsm_tab;               // flat transition table (HR_CFG_FSM_TABLE), or null
    uint32_t launch_seq;             // launches since the job started
    uint64_t shadow_bytes;           // live shadow memory
    std::vector<hr_race> carried;    // global races recovered before a shadow clear
};

// Bytes of the counter words at the start of a context's counter-and-ring
// allocation (the ring follows, 256-byte aligned).
constexpr size_t HR_CTR_BYTES = (HR_CTR_WORDS * sizeof(uint32_t) + 255) / 256 * 256;

hipStream_t hr_stream(hr_ctx c, void* stream);
// A coalescing width: a power of two in 2..64.
inline bool hr_coalesce_width_ok(uint32_t w) { return w >= 2 && w <= 64 && (w & (w - 1)) == 0; }
// Apply the defaults of hr_config and check its ranges (false: invalid).
bool hr_config_normalize(const hr_config* cfg, hr_config* out);
// The hooks' environment of a normalized configuration over the given ring,
// counters and debug counters, at launch number launch_seq.
hr_env hr_env_of(const hr_config& cfg, hr_race_rec* ring, uint32_t* ctr,
                 unsigned long long* count, uint32_t launch_seq, hr_access_rec* log = nullptr);
hr_env hr_make_env(hr_ctx c);
void hr_fill_args(hr_ctx c, hr_kargs* a);
// A region usable through kernel arguments (id < HR_MAX_REGIONS), registered
// for `data` and holding at least min_elems elements.
bool hr_region_ok(hr_ctx c, uint32_t r, const void* data, size_t min_elems);
// Allocate `words` cleared shadow words as a new allocation.
hr_status hr_new_alloc(hr_ctx c, size_t words, uint32_t* alloc_out);
uint32_t hr_new_region(hr_ctx c, const void* data, size_t elems, uint64_t* shadow, uint32_t alloc);
// Shadow words of a region (tiles' padding included).
size_t hr_region_words(const hr_region& r);
void hr_free_alloc(hr_ctx c, uint32_t alloc);
hipError_t hr_fill64(uint64_t* p, size_t n, hipStream_t s);
hipError_t hr_fill32(uint32_t* p, size_t n, hipStream_t s);
// Sort race records by key (space, region, block if LDS, index) and keep
// the first of each key, in place; returns the number kept.
size_t hr_sort_unique(hr_race* recs, size_t n);
// Append a scanned record to ring[] for every race-state word among the
// shadow words [first, first + n) of a region (4-byte words when word4),
// taking slots from *count; ring must have room for n more records.  With
// ring null the race words are only counted in *count.
// rows / lay: the region's map (row-major when lay is zero), which turns a
// word's offset back into its element index.
hipError_t hr_scan_races_dev(const uint64_t* sh, size_t n, size_t first, bool word4,
                             uint32_t region, hr_race_rec* ring, uint32_t* count, hipStream_t s,
                             uint32_t rows = 0, const hr_lay& lay = hr_lay{});

// Shape checks and derived sizes of one job (hr_instance); fills blocks (and
// threads for jacobi), the element counts of its two monitored buffers and
// the LDS bytes of one work item of the batched and serving executors.
bool hr_instance_shape(hr_instance& in, size_t elems[2], size_t* lds_bytes);

// The checked kernels of the workloads with prepared kernel arguments (the
// regions are not validated here; the hr_*_check entries do that).
hr_status hr_launch_reduce(const hr_kargs& a, uint32_t r_in, uint32_t r_out, const int32_t* in_dev,
                           int32_t* out_dev, uint32_t n, uint32_t threads, uint32_t blocks,
                           int32_t drop, hipStream_t s);
hr_status hr_launch_jacobi(const hr_kargs& a, uint32_t r_old, uint32_t r_new,
                           const float* u_old_dev, float* u_new_dev, uint32_t ny, uint32_t nx,
                           const int32_t* seed_dev, hipStream_t s);
hr_status hr_launch_labelprop(const hr_kargs& a, uint32_t r_label, uint32_t r_row_ptr,
                              uint32_t r_col, int32_t* label_dev, const int32_t* row_ptr_dev,
                              const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                              uint32_t tpb, hipStream_t s);

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
