// hr_job_run_static: the serial path for one job (hr_job_run) without any
// allocation.  Its counters, report ring and shadow words live in one
// file-scope device array of fixed size, so a caller that may not allocate
// device memory can still check a job.
//
// Host code never passes the array's name to a kernel or a copy: in host code
// that name is only a stand-in for the symbol.  The array's device address
// is looked up once per device with hipGetSymbolAddress and kept; every use
// below goes through that address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "hr.h"
#include "hr_internal.h"

namespace {

// Byte offsets inside the scratch array.
constexpr size_t OFF_CTR = 0;                          // HR_CTR_WORDS uint32
constexpr size_t OFF_COUNT = 2048;                     // HR_COUNT_SLOTS uint64
constexpr size_t OFF_SCAN = 4096;                      // one uint32: scan slot counter
constexpr size_t OFF_RING = 8192;                      // HR_STATIC_RING_RECORDS records
constexpr size_t OFF_SHADOW = OFF_RING + (size_t)HR_STATIC_RING_RECORDS * sizeof(hr_race_rec);

static_assert(HR_CTR_WORDS * sizeof(uint32_t) <= OFF_COUNT - OFF_CTR, "counter words fit");
static_assert(HR_COUNT_SLOTS * sizeof(uint64_t) <= OFF_SCAN - OFF_COUNT, "count slots fit");
static_assert(OFF_SHADOW % 256 == 0, "shadow words start on a 256-byte boundary");
static_assert(OFF_SHADOW + (size_t)HR_STATIC_SHADOW_WORDS * 8 <= HR_STATIC_SCRATCH_BYTES,
              "shadow words fit");

// The scratch memory: one copy per device, resident while the process lives.
static __device__ __align__(256) uint64_t scratch[HR_STATIC_SCRATCH_BYTES / 8];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;                    // serialises calls of this process
uint8_t* g_base[MAX_DEVICES] = {};    // device address of scratch, per device

// The current device's copy of the scratch array (looked up on the first call
// on that device, with that device current).  Called under g_lock.
hr_status scratch_base(uint8_t** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HR_E_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return HR_E_INVAL;
    if (!g_base[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HR_E_HIP;
        g_base[dev] = (uint8_t*)p;
    }
    *out = g_base[dev];
    return HR_OK;
}

}  // namespace

extern "C" hr_status hr_job_run_static(const hr_instance* inst, const hr_config* cfg,
                                       hr_race* out, size_t cap, size_t* n_out, void* stream)
{
    if (!inst || !n_out) return HR_E_INVAL;
    hr_instance in = *inst;
    size_t el[2] = {0, 0}, lds = 0;
    if (!hr_instance_shape(in, el, &lds)) return HR_E_INVAL;
    hr_config k;
    if (!hr_config_normalize(cfg, &k) ||
        (k.flags & (HR_CFG_WORD4 | HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE)))
        return HR_E_INVAL;
    k.ring_capacity = std::min<uint32_t>(k.ring_capacity, HR_STATIC_RING_RECORDS);
    if (el[0] + el[1] > HR_STATIC_SHADOW_WORDS) return HR_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;

    std::lock_guard<std::mutex> guard(g_lock);
    uint8_t* base = nullptr;
    const hr_status bs = scratch_base(&base);
    if (bs != HR_OK) return bs;
    uint32_t* ctr = (uint32_t*)(base + OFF_CTR);
    unsigned long long* count = (unsigned long long*)(base + OFF_COUNT);
    uint32_t* scan_n = (uint32_t*)(base + OFF_SCAN);
    hr_race_rec* ring = (hr_race_rec*)(base + OFF_RING);
    uint64_t* sh[2] = {(uint64_t*)(base + OFF_SHADOW), (uint64_t*)(base + OFF_SHADOW) + el[0]};

    // The previous call's contents stay in the array: start from zero.
    HR_HIP_CHECK(hr_fill32(ctr, HR_CTR_WORDS, s));
    HR_HIP_CHECK(hr_fill64((uint64_t*)count, HR_COUNT_SLOTS, s));
    HR_HIP_CHECK(hr_fill64(sh[0], el[0] + el[1], s));

    hr_kargs a{};
    for (int r = 0; r < 2; ++r) {
        if (!el[r]) continue;
        a.shadow[r] = sh[r];
        a.n_elems[r] = el[r];
        a.data[r] = const_cast<void*>(in.data[r]);
    }
    // One launch per phase; a job has at most 2^9 phases, so its launch
    // epochs never wrap and the shadow needs no clear in between.
    for (uint32_t p = 0; p < in.phases; ++p) {
        a.env = hr_env_of(k, ring, ctr, count, p);
        hr_status st;
        switch (in.pattern) {
        case HR_PAT_REDUCE:
            st = hr_launch_reduce(a, 0, 1, (const int32_t*)in.data[0], (int32_t*)in.data[1], in.n,
                                  in.threads, in.blocks, in.drop, s);
            break;
        case HR_PAT_JACOBI: {
            const uint32_t o = p & 1u;
            st = hr_launch_jacobi(a, o, 1u - o, (const float*)in.data[o],
                                  (float*)const_cast<void*>(in.data[1 - o]), in.ny, in.n,
                                  (const int32_t*)in.data[2], s);
            break;
        }
        default:
            st = hr_launch_labelprop(a, 0, UINT32_MAX, UINT32_MAX,
                                     (int32_t*)const_cast<void*>(in.data[0]),
                                     (const int32_t*)in.data[1], (const int32_t*)in.data[2],
                                     (const uint8_t*)in.data[3], in.n, in.threads, s);
            break;
        }
        if (st != HR_OK) return st;
    }

    // The report, as hr_report: warnings, ring records, and when records are
    // missing the global races recovered from the sticky race words.
    HR_HIP_CHECK(hipStreamSynchronize(s));
    uint32_t hf[2] = {0, 0};   // HR_CTR_HEAD, HR_CTR_FLAGS
    HR_HIP_CHECK(hipMemcpy(hf, ctr, sizeof(hf), hipMemcpyDeviceToHost));
    const uint32_t head = hf[HR_CTR_HEAD], flags = hf[HR_CTR_FLAGS];
    int warn = 0;
    if (flags & HR_DEVF_CLOCK) warn |= HR_W_CLOCK_OVERFLOW;
    if (flags & HR_DEVF_RANGE) warn |= HR_W_OUT_OF_RANGE;
    if (flags & HR_DEVF_STALL) warn |= HR_W_STALLED;
    if (flags & HR_DEVF_LIMIT) warn |= HR_W_REPORT_LIMITED;
    if (flags & HR_DEVF_FOLD) warn |= HR_W_FOLDED;
    if (flags & HR_DEVF_MASK) warn |= HR_W_PARTIAL_BARRIER;
    if (head > k.ring_capacity) warn |= HR_W_RING_OVERFLOW;
    const size_t n_ring = std::min(head, k.ring_capacity);
    const bool scan = head > k.ring_capacity || (flags & HR_DEVF_LIMIT);
    size_t n_scan = 0;
    if (scan) {   // count the race words first, to size the result
        HR_HIP_CHECK(hr_fill32(scan_n, 1, s));
        for (uint32_t r = 0; r < 2; ++r)
            HR_HIP_CHECK(hr_scan_races_dev(sh[r], el[r], 0, false, r, nullptr, scan_n, s));
        HR_HIP_CHECK(hipStreamSynchronize(s));
        uint32_t cnt = 0;
        HR_HIP_CHECK(hipMemcpy(&cnt, scan_n, sizeof(cnt), hipMemcpyDeviceToHost));
        n_scan = cnt;
    }
    const size_t raw = n_ring + n_scan;
    if (raw > cap || (raw && !out)) {
        *n_out = raw;
        return HR_E_INVAL;
    }
    if (n_ring)
        HR_HIP_CHECK(hipMemcpy(out, ring, sizeof(hr_race) * n_ring, hipMemcpyDeviceToHost));
    size_t m = n_ring;
    if (scan) {
        // The ring's records are on the host now, so its slots take the
        // scanned records, one chunk of at most ring_capacity words at a time
        // (a chunk holds at most that many race words).
        const size_t chunk = k.ring_capacity;
        for (uint32_t r = 0; r < 2; ++r) {
            for (size_t first = 0; first < el[r]; first += chunk) {
                HR_HIP_CHECK(hr_fill32(scan_n, 1, s));
                HR_HIP_CHECK(hr_scan_races_dev(sh[r], std::min(chunk, el[r] - first), first, false,
                                               r, ring, scan_n, s));
                HR_HIP_CHECK(hipStreamSynchronize(s));
                uint32_t cnt = 0;
                HR_HIP_CHECK(hipMemcpy(&cnt, scan_n, sizeof(cnt), hipMemcpyDeviceToHost));
                if (cnt > chunk || m + cnt > raw) return HR_E_STATE;   // cannot happen
                if (cnt)
                    HR_HIP_CHECK(hipMemcpy(out + m, ring, sizeof(hr_race) * cnt,
                                           hipMemcpyDeviceToHost));
                m += cnt;
            }
        }
    }
    *n_out = hr_sort_unique(out, m);
    return (hr_status)warn;
}
