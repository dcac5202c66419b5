// Host runtime of the race checker: contexts, shadow regions, launch epochs
// and the race report.  See hr.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "hr.h"
#include "hr_device.h"
#include "hr_internal.h"

namespace {

__global__ void k_fill64(uint64_t* __restrict__ p, size_t n, uint64_t v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill32(uint32_t* __restrict__ p, size_t n, uint32_t v)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// The launch-boundary clear of 4-byte words, two per 8-byte unit: back to
// the initial state, except that while some race record is missing from the
// ring (it overflowed, or a call site reached its record limit; read on the
// device) a word in the race state keeps it for the report's scan.
__global__ void k_clear_word4(uint64_t* __restrict__ p, size_t n, const uint32_t* __restrict__ ctr,
                              uint32_t ring_cap)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    if (ctr[HR_CTR_HEAD] <= ring_cap && !(ctr[HR_CTR_FLAGS] & HR_DEVF_LIMIT)) {
        for (; i < n; i += stride) p[i] = 0;
        return;
    }
    for (; i < n; i += stride) {
        const uint64_t v = p[i];
        const uint64_t lo = (uint32_t)v == hr::T_RACE ? hr::T_RACE : 0u;
        const uint64_t hi = (uint32_t)(v >> 32) == hr::T_RACE ? hr::T_RACE : 0u;
        p[i] = lo | (hi << 32);
    }
}

hr_status clear_shadows(hr_ctx c, hipStream_t s)
{
    for (const hr_alloc& al : c->allocs)
        if (al.live && hr_fill64(al.mem, al.words, s) != hipSuccess) return HR_E_HIP;
    return HR_OK;
}

// The global races among n shadow words: each word in the race state is
// appended to ring[] as a scanned record (only its key is valid) at the
// index taken from *count, or only counted when ring is null.  The caller
// sizes ring for every word it scans.
// The words are at offsets first .. first + n - 1 of the region's shadow;
// rows and lay give the region's map back to element indices.
__global__ void k_scan_races(const uint64_t* __restrict__ sh, size_t n, size_t first,
                             uint32_t word4, uint32_t region, hr_race_rec* __restrict__ ring,
                             uint32_t* __restrict__ count, uint32_t rows, hr_lay lay)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        const size_t o = first + i;
        const bool race = word4 ? ((const uint32_t*)sh)[o] == hr::T_RACE
                                : (sh[o] & hr::g::TAG_M) == hr::T_RACE;
        const uint64_t e = hr_lay_index(lay, rows, o);
        if (!race || e == UINT64_MAX) continue;
        const uint32_t slot =
            __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!ring) continue;
        uint4* p = reinterpret_cast<uint4*>(ring + slot);
        p[0] = make_uint4(0u, region, 0xFFFFFFFFu, 0xFFFFFFFFu);
        p[1] = make_uint4((uint32_t)e, (uint32_t)(e >> 32), 0u, 0u);
        p[2] = make_uint4(0u, 0u, 0xFFFFFFFFu, HR_RACE_SCANNED);
    }
}

}  // namespace

namespace {
uint32_t key_block(const hr_race& r) { return r.space == HR_LDS ? r.block : 0u; }

bool key_less(const hr_race& a, const hr_race& b)
{
    if (a.space != b.space) return a.space < b.space;
    if (a.region != b.region) return a.region < b.region;
    if (key_block(a) != key_block(b)) return key_block(a) < key_block(b);
    if (a.index != b.index) return a.index < b.index;
    return a.launch < b.launch;
}

bool key_same(const hr_race& a, const hr_race& b)
{
    return a.space == b.space && a.region == b.region && key_block(a) == key_block(b) &&
           a.index == b.index;
}
}  // namespace

size_t hr_sort_unique(hr_race* recs, size_t n)
{
    std::sort(recs, recs + n, key_less);
    size_t m = 0;
    for (size_t i = 0; i < n; ++i)
        if (m == 0 || !key_same(recs[m - 1], recs[i])) recs[m++] = recs[i];
    return m;
}

hipError_t hr_scan_races_dev(const uint64_t* sh, size_t n, size_t first, bool word4,
                             uint32_t region, hr_race_rec* ring, uint32_t* count, hipStream_t s,
                             uint32_t rows, const hr_lay& lay)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_scan_races, dim3((unsigned)blocks), dim3(256), 0, s, sh, n, first,
                       word4 ? 1u : 0u, region, ring, count, rows, lay);
    return hipGetLastError();
}

// Clears run as kernels rather than hipMemsetAsync so the calls stay safe
// inside a captured HIP graph.
hipError_t hr_fill64(uint64_t* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
    (void)hipGetLastError();   // drop stale errors of unrelated earlier calls
    hipLaunchKernelGGL(k_fill64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, 0ull);
    return hipGetLastError();
}

hipError_t hr_fill32(uint32_t* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, 0u);
    return hipGetLastError();
}

hipStream_t hr_stream(hr_ctx c, void* stream)
{
    return stream ? (hipStream_t)stream : c->stream;
}

hr_env hr_env_of(const hr_config& cfg, hr_race_rec* ring, uint32_t* ctr,
                 unsigned long long* count, uint32_t launch_seq, hr_access_rec* log)
{
    hr_env e{};
    e.ring = ring;
    e.ctr = ctr;
    e.count = (cfg.flags & (HR_CFG_COUNT_CHECKS | HR_CFG_ACCESS_LOG)) ? count : nullptr;
    e.log = (cfg.flags & HR_CFG_ACCESS_LOG) ? log : nullptr;
    e.log_cap = e.log ? cfg.log_capacity : 0u;
    e.ring_cap = cfg.ring_capacity;
    e.launch = launch_seq & ((1u << hr::g::LAUNCH_BITS) - 1);
    e.launch_seq = launch_seq;
    e.bc_max = (1u << cfg.bc_bits) - 1;
    e.wc_max = (1u << cfg.wc_bits) - 1;
    e.group = (cfg.flags & HR_CFG_WAVE_GROUPING) ? cfg.coalesce_width : 0u;
    e.site_limit = cfg.site_limit;
    e.wave_bits = cfg.wave_bits;
    e.nested = (cfg.flags & HR_CFG_NESTED_TILES) ? 1u : 0u;
    e.word4 = (cfg.flags & HR_CFG_WORD4)
                  ? hr::c::layout(cfg.wc_bits, cfg.bc_bits, cfg.thread_bits)
                  : 0u;
    return e;
}

hr_env hr_make_env(hr_ctx c)
{
    return hr_env_of(c->cfg, c->ring, c->ctr, c->count, c->launch_seq, c->log);
}

void hr_fill_args(hr_ctx c, hr_kargs* a)
{
    *a = hr_kargs{};
    a->env = hr_make_env(c);
    const uint32_t n = (uint32_t)std::min<size_t>(c->reg.size(), HR_MAX_REGIONS);
    for (uint32_t r = 0; r < n; ++r) {
        if (!c->reg[r].live) continue;
        a->shadow[r] = c->reg[r].monitored ? c->reg[r].shadow : nullptr;
        a->n_elems[r] = c->reg[r].elems;
        a->data[r] = const_cast<void*>(c->reg[r].data);
        a->lay[r] = c->reg[r].lay;
    }
}

bool hr_region_ok(hr_ctx c, uint32_t r, const void* data, size_t min_elems)
{
    return r < HR_MAX_REGIONS && r < c->reg.size() && c->reg[r].live && c->reg[r].data == data &&
           c->reg[r].elems >= min_elems;
}

hr_status hr_new_alloc(hr_ctx c, size_t words, uint32_t* alloc_out)
{
    const uint64_t bytes = (uint64_t)words * 8u;
    if (c->cfg.shadow_budget && c->shadow_bytes + bytes > c->cfg.shadow_budget) return HR_E_NOMEM;
    uint64_t* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return HR_E_NOMEM;
    if (hr_fill64(mem, words, c->stream) != hipSuccess) {
        (void)hipFree(mem);
        return HR_E_HIP;
    }
    c->allocs.push_back(hr_alloc{mem, words, true});
    c->shadow_bytes += bytes;
    *alloc_out = (uint32_t)(c->allocs.size() - 1);
    return HR_OK;
}

uint32_t hr_new_region(hr_ctx c, const void* data, size_t elems, uint64_t* shadow, uint32_t alloc)
{
    c->reg.push_back(hr_region{data, elems, shadow, alloc, true, true});
    return (uint32_t)(c->reg.size() - 1);
}

size_t hr_region_words(const hr_region& r)
{
    return hr_lay_words(r.lay, r.rows, r.elems);
}

void hr_free_alloc(hr_ctx c, uint32_t alloc)
{
    hr_alloc& al = c->allocs[alloc];
    if (!al.live) return;
    (void)hipFree(al.mem);
    al.live = false;
    c->shadow_bytes -= (uint64_t)al.words * 8u;
    for (hr_region& r : c->reg)
        if (r.alloc == alloc) r.live = false;
}

// The flat transition table of the global-word machine, built at compile
// time from its bit logic (hr::g::make_step_table).
static constexpr hr::g::step_table FSM_TABLE = hr::g::make_step_table();
static_assert(hr::g::step_table_consistent(), "the flat table must rebuild hr::g::step");

bool hr_config_normalize(const hr_config* cfg, hr_config* out)
{
    hr_config k = {};
    if (cfg) k = *cfg;
    const bool word4 = (k.flags & HR_CFG_WORD4) != 0;
    const bool nested = (k.flags & HR_CFG_NESTED_TILES) != 0;
    if (nested) {
        // tiles of 2^wave_bits lanes inside whole waves; the nested words'
        // clock fields hold 5 and 4 bits, and the flat options do not apply
        if (k.wave_bits < 1 || k.wave_bits > 5 || word4 || (k.flags & HR_CFG_WAVE_GROUPING))
            return false;
        if (k.bc_bits == 0) k.bc_bits = 5;
        if (k.wc_bits == 0) k.wc_bits = 4;
        if (k.bc_bits > 5 || k.wc_bits > 4) return false;
    }
    if (k.ring_capacity == 0) k.ring_capacity = 65536;
    if (k.bc_bits == 0) k.bc_bits = word4 ? 2 : 8;
    if (k.wc_bits == 0) k.wc_bits = word4 ? 1 : 6;
    if (k.thread_bits == 0) k.thread_bits = word4 ? 8 : 10;
    if (k.bc_bits > 8 || k.wc_bits > 6 || k.ring_capacity > (1u << 26)) return false;
    if (k.thread_bits > 10 || (!word4 && k.thread_bits != 10)) return false;
    if (k.flags & HR_CFG_FSM_TABLE_LDS) k.flags |= HR_CFG_FSM_TABLE;
    if (k.flags & ~(HR_CFG_COUNT_CHECKS | HR_CFG_WAVE_GROUPING | HR_CFG_WORD4 |
                    HR_CFG_ACCESS_LOG | HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE |
                    HR_CFG_FSM_TABLE_LDS))
        return false;
    if ((k.flags & HR_CFG_FSM_TABLE) &&
        (k.flags & (HR_CFG_WORD4 | HR_CFG_NESTED_TILES | HR_CFG_ACCESS_LOG)))
        return false;
    if (k.flags & HR_CFG_ACCESS_LOG) {
        if (k.log_capacity == 0) k.log_capacity = 1u << 20;
        if (k.log_capacity > (1u << 28)) return false;
    } else if (k.log_capacity) {
        return false;   // a log size without the log
    }
    if (k.wave_bits == 0) k.wave_bits = 6;
    if (k.wave_bits > 6) return false;
    if (k.flags & HR_CFG_WAVE_GROUPING) {
        if (k.coalesce_width == 0) k.coalesce_width = 64;
        if (!hr_coalesce_width_ok(k.coalesce_width)) return false;
    } else if (k.coalesce_width) {
        return false;   // a width without grouping
    }
    *out = k;
    return true;
}

extern "C" hr_status hr_ctx_create(hr_ctx* out, const hr_config* cfg, void* stream)
{
    if (!out) return HR_E_INVAL;
    *out = nullptr;
    hr_config k;
    if (!hr_config_normalize(cfg, &k)) return HR_E_INVAL;
    hr_ctx c = new (std::nothrow) hr_ctx_s();
    if (!c) return HR_E_NOMEM;
    c->cfg = k;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return HR_E_HIP;
    }
    if (hipMalloc(&c->ctr, HR_CTR_BYTES + sizeof(hr_race_rec) * (size_t)k.ring_capacity) !=
        hipSuccess) {
        hr_ctx_destroy(c);
        return HR_E_NOMEM;
    }
    c->ring = (hr_race_rec*)((uint8_t*)c->ctr + HR_CTR_BYTES);
    if (hipMalloc(&c->count, sizeof(unsigned long long) * HR_COUNT_SLOTS) != hipSuccess ||
        ((k.flags & HR_CFG_ACCESS_LOG) &&
         hipMalloc(&c->log, sizeof(hr_access_rec) * (size_t)k.log_capacity) != hipSuccess) ||
        ((k.flags & HR_CFG_FSM_TABLE) && hipMalloc(&c->fsm_tab, sizeof(FSM_TABLE)) != hipSuccess)) {
        hr_ctx_destroy(c);
        return HR_E_NOMEM;
    }
    if (c->fsm_tab && hipMemcpy(c->fsm_tab, FSM_TABLE.e, sizeof(FSM_TABLE),
                                hipMemcpyHostToDevice) != hipSuccess) {
        hr_ctx_destroy(c);
        return HR_E_HIP;
    }
    if (hr_fill32(c->ctr, HR_CTR_WORDS, c->stream) != hipSuccess ||
        hr_fill64((uint64_t*)c->count, HR_COUNT_SLOTS, c->stream) != hipSuccess) {
        hr_ctx_destroy(c);
        return HR_E_HIP;
    }
    *out = c;
    return HR_OK;
}

extern "C" hr_status hr_ctx_destroy(hr_ctx c)
{
    if (!c) return HR_E_INVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    for (hr_alloc& al : c->allocs)
        if (al.live) (void)hipFree(al.mem);
    if (c->ctr) (void)hipFree(c->ctr);   // the ring's memory too
    if (c->count) (void)hipFree(c->count);
    if (c->log) (void)hipFree(c->log);
    if (c->fsm_tab) (void)hipFree(c->fsm_tab);
    delete c;
    return e == hipSuccess ? HR_OK : HR_E_HIP;
}

extern "C" hr_status hr_shadow_alloc(hr_ctx c, const void* data_dev, size_t bytes,
                                     uint32_t elem_bytes, uint32_t* region_out)
{
    if (!c || !region_out || elem_bytes != 4 || bytes == 0 || bytes % 4 != 0) return HR_E_INVAL;
    if (c->reg.size() >= (1u << 24)) return HR_E_INVAL;
    const size_t elems = bytes / 4;
    uint32_t alloc = 0;
    const size_t words = (c->cfg.flags & HR_CFG_WORD4) ? (elems + 1) / 2 : elems;
    const hr_status st = hr_new_alloc(c, words, &alloc);
    if (st != HR_OK) return st;
    *region_out = hr_new_region(c, data_dev, elems, c->allocs[alloc].mem, alloc);
    return HR_OK;
}

extern "C" hr_status hr_shadow_alloc_2d(hr_ctx c, const void* data_dev, uint32_t rows,
                                        uint32_t cols, uint32_t elem_bytes, uint32_t tile_w_log2,
                                        uint32_t tile_h_log2, uint32_t* region_out)
{
    if (!c || !region_out || elem_bytes != 4 || rows == 0 || cols == 0) return HR_E_INVAL;
    if (tile_w_log2 > HR_TILE_LOG2_MAX || tile_h_log2 > HR_TILE_LOG2_MAX ||
        tile_w_log2 + tile_h_log2 > 2 * HR_TILE_LOG2_MAX)
        return HR_E_INVAL;
    if (c->reg.size() >= (1u << 24)) return HR_E_INVAL;
    hr_lay L{cols, (cols + (1u << tile_w_log2) - 1u) >> tile_w_log2, tile_w_log2, tile_h_log2};
    if ((tile_w_log2 | tile_h_log2) == 0) L = hr_lay{};   // row-major: the identity map
    const size_t elems = (size_t)rows * cols;
    const size_t lw = hr_lay_words(L, rows, elems);
    const size_t words = (c->cfg.flags & HR_CFG_WORD4) ? (lw + 1) / 2 : lw;
    uint32_t alloc = 0;
    const hr_status st = hr_new_alloc(c, words, &alloc);
    if (st != HR_OK) return st;
    *region_out = hr_new_region(c, data_dev, elems, c->allocs[alloc].mem, alloc);
    c->reg[*region_out].lay = L;
    c->reg[*region_out].rows = rows;
    return HR_OK;
}

extern "C" hr_status hr_shadow_free(hr_ctx c, uint32_t region)
{
    if (!c || region >= c->reg.size() || !c->reg[region].live) return HR_E_INVAL;
    const uint32_t alloc = c->reg[region].alloc;
    for (const hr_region& r : c->reg)
        if (r.live && r.alloc == alloc && &r != &c->reg[region]) return HR_E_STATE;   // shared arena
    if (hipStreamSynchronize(c->stream) != hipSuccess) return HR_E_HIP;
    hr_free_alloc(c, alloc);
    return HR_OK;
}

extern "C" hr_status hr_dev_args(hr_ctx c, void* out, size_t cap, size_t* size_out)
{
    if (!c) return HR_E_INVAL;
    if (size_out) *size_out = sizeof(hr_kargs);
    if (!out || cap < sizeof(hr_kargs)) return HR_E_INVAL;
    hr_fill_args(c, (hr_kargs*)out);
    return HR_OK;
}

static hr_race scanned_race(uint32_t region, size_t index)
{
    hr_race x = {};
    x.space = HR_GLOBAL;
    x.region = region;
    x.block = 0xFFFFFFFFu;
    x.launch = 0xFFFFFFFFu;
    x.index = index;
    x.tid = 0xFFFFFFFFu;
    x.flags = HR_RACE_SCANNED;
    return x;
}

// The global races held in the sticky race words of every live region.
static hr_status scan_races(hr_ctx c, std::vector<hr_race>& out)
{
    const bool word4 = (c->cfg.flags & HR_CFG_WORD4) != 0;
    for (uint32_t r = 0; r < c->reg.size(); ++r) {
        if (!c->reg[r].live) continue;
        const hr_region& g = c->reg[r];
        const size_t words = hr_region_words(g);
        if (word4) {
            std::vector<uint32_t> sh(words);
            if (hipMemcpy(sh.data(), g.shadow, sizeof(uint32_t) * sh.size(),
                          hipMemcpyDeviceToHost) != hipSuccess)
                return HR_E_HIP;
            for (size_t i = 0; i < sh.size(); ++i)
                if (sh[i] == hr::T_RACE && hr_lay_index(g.lay, g.rows, i) != UINT64_MAX)
                    out.push_back(scanned_race(r, hr_lay_index(g.lay, g.rows, i)));
            continue;
        }
        std::vector<uint64_t> sh(words);
        if (hipMemcpy(sh.data(), g.shadow, sizeof(uint64_t) * sh.size(),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return HR_E_HIP;
        for (size_t i = 0; i < sh.size(); ++i) {
            if ((sh[i] & hr::g::TAG_M) == hr::T_RACE && hr_lay_index(g.lay, g.rows, i) != UINT64_MAX)
                out.push_back(scanned_race(r, hr_lay_index(g.lay, g.rows, i)));
        }
    }
    return HR_OK;
}

extern "C" hr_status hr_kernel_end(hr_ctx c, void* stream)
{
    if (!c) return HR_E_INVAL;
    c->launch_seq += 1;
    if (c->cfg.flags & HR_CFG_WORD4) {
        // No launch field: every boundary returns the words to INIT.
        hipStream_t s = hr_stream(c, stream);
        for (const hr_alloc& al : c->allocs) {
            if (!al.live || al.words == 0) continue;
            const size_t blocks = std::min<size_t>((al.words + 255) / 256, 8192);
            HR_LAUNCH(k_clear_word4, dim3((unsigned)blocks), dim3(256), 0, s, al.mem, al.words,
                      c->ctr, c->cfg.ring_capacity);
        }
        return HR_OK;
    }
    // The launch epoch in a shadow word has 9 bits: before it wraps, return
    // every word to the initial state.  Exact: all earlier accesses happen
    // before all later ones, and the races found so far are in the ring.
    // If the ring has overflowed or a call site reached its record limit,
    // the races whose records are missing live only in the race words, so
    // they are recovered before the clear and carried to the report.
    if ((c->launch_seq & ((1u << hr::g::LAUNCH_BITS) - 1)) == 0) {
        hipStream_t s = hr_stream(c, stream);
        uint32_t hf[2] = {0, 0};   // HR_CTR_HEAD, HR_CTR_FLAGS
        if (hipMemcpyAsync(hf, c->ctr, sizeof(hf), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return HR_E_HIP;
        if (hf[HR_CTR_HEAD] > c->cfg.ring_capacity || (hf[HR_CTR_FLAGS] & HR_DEVF_LIMIT)) {
            const hr_status st = scan_races(c, c->carried);
            if (st != HR_OK) return st;
        }
        return clear_shadows(c, s);
    }
    return HR_OK;
}

extern "C" hr_status hr_reset(hr_ctx c, void* stream)
{
    if (!c) return HR_E_INVAL;
    hipStream_t s = hr_stream(c, stream);
    hr_status st = clear_shadows(c, s);
    if (st != HR_OK) return st;
    if (hr_fill32(c->ctr, HR_CTR_WORDS, s) != hipSuccess) return HR_E_HIP;
    if (hr_fill64((uint64_t*)c->count, HR_COUNT_SLOTS, s) != hipSuccess) return HR_E_HIP;
    c->launch_seq = 0;
    c->carried.clear();
    return HR_OK;
}

extern "C" hr_status hr_region_enable(hr_ctx c, uint32_t region, uint32_t on)
{
    if (!c || region >= c->reg.size() || !c->reg[region].live) return HR_E_INVAL;
    c->reg[region].monitored = on != 0;
    return HR_OK;
}

extern "C" hr_status hr_report(hr_ctx c, hr_race* out, size_t cap, size_t* n_out, void* stream)
{
    if (!c || !n_out) return HR_E_INVAL;
    hipStream_t s = hr_stream(c, stream);
    // One copy, after the stream's work, reads the counters and as many ring
    // records as the last report found (at least 64); a second copy reads
    // the rest when there are more.
    const uint32_t pre = std::min(c->cfg.ring_capacity, std::max(64u, c->last_head));
    std::vector<uint8_t> buf(HR_CTR_BYTES + sizeof(hr_race_rec) * (size_t)pre);
    if (hipMemcpyAsync(buf.data(), c->ctr, buf.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return HR_E_HIP;
    uint32_t ctr[HR_CTR_SITES];
    std::memcpy(ctr, buf.data(), sizeof(ctr));
    const uint32_t head = ctr[HR_CTR_HEAD];
    const uint32_t n_ring = std::min(head, c->cfg.ring_capacity);
    c->last_head = n_ring;
    std::vector<hr_race> recs(n_ring);
    const uint32_t have = std::min(n_ring, pre);
    if (have) std::memcpy(recs.data(), buf.data() + HR_CTR_BYTES, sizeof(hr_race) * have);
    if (n_ring > have &&
        hipMemcpy(recs.data() + have, c->ring + have, sizeof(hr_race) * (n_ring - have),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return HR_E_HIP;
    int warn = 0;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_CLOCK) warn |= HR_W_CLOCK_OVERFLOW;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_RANGE) warn |= HR_W_OUT_OF_RANGE;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_STALL) warn |= HR_W_STALLED;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_LIMIT) warn |= HR_W_REPORT_LIMITED;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_FOLD) warn |= HR_W_FOLDED;
    if (ctr[HR_CTR_FLAGS] & HR_DEVF_MASK) warn |= HR_W_PARTIAL_BARRIER;
    if (head > c->cfg.ring_capacity) warn |= HR_W_RING_OVERFLOW;
    if (head > c->cfg.ring_capacity || (ctr[HR_CTR_FLAGS] & HR_DEVF_LIMIT)) {
        // Race records are missing (ring overflow, or a site past its record
        // limit): race states are sticky in global shadow memory, so the
        // global part of the flagged set is recovered from it exactly (and
        // from the races carried over a shadow clear).
        const hr_status st = scan_races(c, recs);
        if (st != HR_OK) return st;
        recs.insert(recs.end(), c->carried.begin(), c->carried.end());
    }
    const size_t n = hr_sort_unique(recs.data(), recs.size());
    *n_out = n;
    if (n > cap || (n && !out)) return HR_E_INVAL;
    std::copy(recs.begin(), recs.begin() + n, out);
    return (hr_status)warn;
}

extern "C" hr_status hr_check_count(hr_ctx c, uint64_t* out, void* stream)
{
    if (!c || !out) return HR_E_INVAL;
    if (hipStreamSynchronize(hr_stream(c, stream)) != hipSuccess) return HR_E_HIP;
    unsigned long long slots[HR_COUNT_SLOTS];
    if (hipMemcpy(slots, c->count, sizeof(slots), hipMemcpyDeviceToHost) != hipSuccess)
        return HR_E_HIP;
    uint64_t sum = 0;
    for (int i = 0; i < HR_COUNT_SLOTS; ++i) sum += slots[i];
    *out = sum;
    return HR_OK;
}

extern "C" hr_status hr_access_log(hr_ctx c, hr_access_rec* out, size_t cap, size_t* n_out,
                                   void* stream)
{
    if (!c || !n_out || !c->log) return HR_E_INVAL;
    if (hipStreamSynchronize(hr_stream(c, stream)) != hipSuccess) return HR_E_HIP;
    uint32_t head = 0;
    if (hipMemcpy(&head, c->ctr + HR_CTR_LOG, sizeof(head), hipMemcpyDeviceToHost) != hipSuccess)
        return HR_E_HIP;
    const size_t n = std::min<size_t>(head, c->cfg.log_capacity);
    *n_out = n;
    if (n > cap || (n && !out)) return HR_E_INVAL;
    if (n && hipMemcpy(out, c->log, sizeof(hr_access_rec) * n, hipMemcpyDeviceToHost) != hipSuccess)
        return HR_E_HIP;
    return head > c->cfg.log_capacity ? HR_W_LOG_TRUNCATED : HR_OK;
}

extern "C" hr_status hr_fsm_step(uint32_t space, uint64_t old, uint32_t kind, uint32_t launch,
                                 uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc,
                                 uint32_t wave_bits, uint64_t* new_out)
{
    if (!new_out || kind > 2 || space > 1 || thread > 1023) return HR_E_INVAL;
    if (wave_bits < 1 || wave_bits > 6) return HR_E_INVAL;
    const uint32_t k = hr::kind_class(kind);
    if (space == HR_GLOBAL) {
        if (block >= hr::g::BLOCK_LIMIT) return HR_E_INVAL;
        *new_out = hr::g::step(old, hr::g::pack_id(launch, block, thread, bc, wc), k,
                               hr::g::group_mask(wave_bits));
    } else {
        *new_out = hr::l::step((uint32_t)old, hr::l::pack_id(thread, bc, wc), k,
                               hr::l::group_mask(wave_bits));
    }
    return HR_OK;
}

extern "C" hr_status hr_fsm_step_table(uint32_t space, uint64_t old, uint32_t kind,
                                       uint32_t launch, uint32_t block, uint32_t thread,
                                       uint32_t bc, uint32_t wc, uint32_t wave_bits,
                                       uint64_t* new_out)
{
    if (!new_out || kind > 2 || space != HR_GLOBAL || thread > 1023) return HR_E_INVAL;
    if (wave_bits < 1 || wave_bits > 6 || block >= hr::g::BLOCK_LIMIT) return HR_E_INVAL;
    *new_out = hr::g::step_tab(FSM_TABLE.e, old, hr::g::pack_id(launch, block, thread, bc, wc),
                               hr::kind_class(kind), hr::g::group_mask(wave_bits));
    return HR_OK;
}

extern "C" hr_status hr_describe(uint32_t space, uint64_t word, uint32_t wave_bits,
                                 hr_summary* out)
{
    if (!out || space > HR_LDS || wave_bits < 1 || wave_bits > 6) return HR_E_INVAL;
    const uint32_t none = UINT32_MAX;
    hr_summary d = {};
    d.launch = d.block = d.bc = d.wave = d.wc = d.thread = none;
    uint32_t tag, cl = 0, cb, cw, bc, wc, th;
    if (space == HR_GLOBAL) {
        namespace g = hr::g;
        tag = (uint32_t)(word & g::TAG_M);
        cl = (uint32_t)(word >> g::CL_SH) & 3u;
        cb = (uint32_t)(word >> g::CB_SH) & 3u;
        cw = (uint32_t)(word >> g::CW_SH) & 3u;
        bc = (uint32_t)(word >> g::BC_SH) & 255u;
        wc = (uint32_t)(word >> g::WC_SH) & 63u;
        th = (uint32_t)(word >> g::TH_SH) & 1023u;
        if (tag > hr::T_ST) return HR_E_INVAL;
        if (tag >= hr::T_MB) d.launch = (uint32_t)(word >> g::LA_SH) & 511u;
        if (tag >= hr::T_MW) d.block = (uint32_t)(word >> g::BL_SH) & (g::BLOCK_LIMIT - 1);
    } else {
        namespace l = hr::l;
        const uint32_t w = (uint32_t)word;
        tag = w & l::TAG_M;
        cb = (w >> l::CB_SH) & 3u;
        cw = (w >> l::CW_SH) & 3u;
        bc = (w >> l::BC_SH) & 255u;
        wc = (w >> l::WC_SH) & 63u;
        th = (w >> l::TH_SH) & 1023u;
        if (tag > hr::T_ST || tag == hr::T_MB) return HR_E_INVAL;
    }
    d.state = tag;
    if (tag >= hr::T_MW) {
        d.class_launch = cl;
        d.bc = bc;
    }
    if (tag == hr::T_MB || tag == hr::T_MW) d.class_block = cb;
    if (tag >= hr::T_MT) {
        d.class_block = cb;
        d.wave = th >> wave_bits;
        d.wc = wc;
    }
    if (tag == hr::T_MW || tag == hr::T_MT) d.class_wave = tag == hr::T_MT ? cw : 0;
    if (tag == hr::T_ST) {
        d.class_wave = cw;
        d.thread = th;
    }
    *out = d;
    return HR_OK;
}

extern "C" hr_status hr_describe_nested(uint32_t space, uint64_t word, uint32_t tile_bits,
                                        hr_summary_nested* out)
{
    if (!out || space > HR_LDS || tile_bits < 1 || tile_bits > 5) return HR_E_INVAL;
    const uint32_t none = UINT32_MAX;
    hr_summary_nested d = {};
    d.launch = d.block = d.bc = d.wave = d.wc = d.tile = d.tc = d.thread = none;
    uint32_t tag, cl = 0, cb, cw, ct, bc, wc, tc, th;
    if (space == HR_GLOBAL) {
        namespace n = hr::n;
        tag = (uint32_t)(word & n::TAG_M);
        cl = (uint32_t)(word >> n::CL_SH) & 3u;
        cb = (uint32_t)(word >> n::CB_SH) & 3u;
        cw = (uint32_t)(word >> n::CW_SH) & 3u;
        ct = (uint32_t)(word >> n::CT_SH) & 3u;
        bc = (uint32_t)(word >> n::BC_SH) & 63u;
        wc = (uint32_t)(word >> n::WC_SH) & 15u;
        tc = (uint32_t)(word >> n::TC_SH) & 15u;
        th = (uint32_t)(word >> n::TH_SH) & 1023u;
        if (tag > hr::T_MTI) return HR_E_INVAL;
        if (tag >= hr::T_MB) d.launch = (uint32_t)(word >> n::LA_SH) & 511u;
        if (tag >= hr::T_MW) d.block = (uint32_t)(word >> n::BL_SH) & (n::BLOCK_LIMIT - 1);
    } else {
        namespace nl = hr::nl;
        const uint32_t w = (uint32_t)word;
        tag = w & nl::TAG_M;
        cb = (w >> nl::CB_SH) & 3u;
        cw = (w >> nl::CW_SH) & 3u;
        ct = (w >> nl::CT_SH) & 3u;
        bc = (w >> nl::BC_SH) & 31u;
        wc = (w >> nl::WC_SH) & 15u;
        tc = (w >> nl::TC_SH) & 15u;
        th = (w >> nl::TH_SH) & 1023u;
        if (tag > hr::T_MTI || tag == hr::T_MB) return HR_E_INVAL;
    }
    // Tag order of the nested machine, from the widest group down: MB
    // (blocks), MW (waves), MTI (tiles of one wave), MT (threads of one
    // tile), ST (one thread).
    const bool mw = tag == hr::T_MW, mti = tag == hr::T_MTI, mt = tag == hr::T_MT,
               st = tag == hr::T_ST;
    d.state = mti ? (uint32_t)HR_S_TILES : tag;
    if (tag == hr::T_MB) d.class_block = cb;
    if (mw || mti || mt || st) {
        d.class_launch = cl;
        d.class_block = cb;
        d.bc = bc;
    }
    if (mti || mt || st) {
        d.class_wave = cw;
        d.wave = th >> 6;
        d.wc = wc;
    }
    if (mt || st) {
        d.class_tile = ct;
        d.tile = th >> tile_bits;
        d.tc = tc;
    }
    if (st) d.thread = th;
    *out = d;
    return HR_OK;
}

static bool word4_widths(uint32_t* wc_bits, uint32_t* bc_bits, uint32_t* thread_bits)
{
    if (*wc_bits == 0) *wc_bits = 1;
    if (*bc_bits == 0) *bc_bits = 2;
    if (*thread_bits == 0) *thread_bits = 8;
    return *wc_bits <= 6 && *bc_bits <= 8 && *thread_bits <= 10;   // the block keeps >= 3 bits
}

extern "C" hr_status hr_fsm_step_word4(uint32_t old, uint32_t kind, uint32_t block,
                                       uint32_t thread, uint32_t bc, uint32_t wc,
                                       uint32_t wave_bits, uint32_t wc_bits, uint32_t bc_bits,
                                       uint32_t thread_bits, uint32_t* new_out)
{
    if (!new_out || kind > 2 || wave_bits < 1 || wave_bits > 6 ||
        !word4_widths(&wc_bits, &bc_bits, &thread_bits) || bc >= (1u << bc_bits) ||
        wc >= (1u << wc_bits) || (old & 31u) >= hr::c::N_STATES)
        return HR_E_INVAL;
    const uint32_t lay = hr::c::layout(wc_bits, bc_bits, thread_bits);
    *new_out = hr::c::step(old, hr::c::pack_id32(block, thread, bc, wc, lay),
                           hr::kind_class(kind), hr::c::group_mask(wave_bits, lay), lay);
    return HR_OK;
}

extern "C" hr_status hr_word4_widen(uint32_t word, uint32_t wc_bits, uint32_t bc_bits,
                                    uint32_t thread_bits, uint64_t* out)
{
    if (!out || !word4_widths(&wc_bits, &bc_bits, &thread_bits) ||
        (word & 31u) >= hr::c::N_STATES)
        return HR_E_INVAL;
    *out = hr::c::widen(word, hr::c::layout(wc_bits, bc_bits, thread_bits));
    return HR_OK;
}

extern "C" hr_status hr_fsm_step_nested(uint32_t space, uint64_t old, uint32_t kind,
                                        uint32_t launch, uint32_t block, uint32_t thread,
                                        uint32_t bc, uint32_t wc, uint32_t tc, uint32_t tile_bits,
                                        uint64_t* new_out)
{
    if (!new_out || kind > 2 || space > 1 || thread > 1023 || tile_bits < 1 || tile_bits > 5)
        return HR_E_INVAL;
    if (block >= hr::n::BLOCK_LIMIT || bc >= hr::n::BC_LIMIT || wc >= hr::n::WC_LIMIT ||
        tc >= hr::n::TC_LIMIT)
        return HR_E_INVAL;
    const uint32_t k = hr::kind_class(kind);
    if (space == HR_GLOBAL)
        *new_out = hr::n::step(old, hr::n::pack_id(launch, block, thread, bc, wc, tc), k,
                               hr::n::tile_mask(tile_bits));
    else
        *new_out = hr::nl::step((uint32_t)old, hr::nl::pack_id(thread, bc, wc, tc), k,
                                hr::nl::tile_mask(tile_bits));
    return HR_OK;
}

extern "C" hr_status hr_fsm_merge_nested(uint64_t x, uint64_t y, uint32_t tile_bits,
                                         uint64_t* out)
{
    if (!out || tile_bits < 1 || tile_bits > 5) return HR_E_INVAL;
    *out = hr::n::merge(x, y, hr::n::tile_mask(tile_bits));
    return HR_OK;
}

extern "C" hr_status hr_fsm_merge(uint64_t x, uint64_t y, uint32_t wave_bits, uint64_t* out)
{
    if (!out || wave_bits < 1 || wave_bits > 6) return HR_E_INVAL;
    *out = hr::g::merge(x, y, hr::g::group_mask(wave_bits));
    return HR_OK;
}
