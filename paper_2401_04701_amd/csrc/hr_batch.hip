// Batched checking: many independent checked jobs ("instances") run to
// completion in one persistent launch, and the serial path that runs one job
// at a time (allocate shadow, launch each phase, report, free).
//
// The persistent launch keeps every worker block resident.  Workers claim
// work items (instance, phase, pack of logical blocks) in queue order from a
// global cursor.  A phase of an instance stands in for one kernel launch of
// that job: an item of phase p waits until every item of phase p-1 of its
// instance has finished, which gives the launch boundary's happens-before edge, and the
// shadow words of the instance carry p as their launch epoch.  Every item
// that phase p waits for sits earlier in the queue and was claimed by a
// resident worker, so the earliest unfinished item always makes progress; a
// bounded wait still guards against a broken queue (HR_W_STALLED).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "hr.h"
#include "hr_bodies.h"
#include "hr_device.h"
#include "hr_exec.h"
#include "hr_internal.h"

namespace {

__device__ __forceinline__ uint64_t claim(uint32_t* cursor, const uint64_t* items, uint32_t n_items)
{
    const uint32_t i = __hip_atomic_fetch_add(cursor, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return i < n_items ? items[i] : ~0ull;
}

// Worker loop.  MIN_WAVES is the occupancy target per SIMD: 4 gives one
// 1024-thread worker per compute unit with up to 128 registers per lane, 8
// gives two workers per compute unit within 64 registers (some values then
// live in scratch).  The autotuner picks between them by measurement.
//
// Thread 0 alone claims items, waits for phases and counts finished items.
// Each of those thread-0 regions sits strictly between two block barriers,
// and every iteration ends with a barrier, so no divergent region spans the
// loop's back edge and every barrier runs with the whole block active.
template <int MIN_WAVES>
__device__ __forceinline__ void batch_loop(const hr_env& base, const hr_inst_dev* __restrict__ insts,
                                           const uint64_t* __restrict__ items, uint32_t n_items,
                                           uint32_t* cursor, uint32_t* done, uint32_t spin_limit)
{
    extern __shared__ uint32_t smem[];
    __shared__ uint64_t s_item;
    __shared__ uint32_t s_go;
    if (threadIdx.x == 0) s_item = claim(cursor, items, n_items);
    __syncthreads();
    for (;;) {
        const uint64_t it = uni64(s_item);
        if (it == ~0ull) break;                         // queue drained: every wave leaves
        const uint32_t ii = (uint32_t)(it >> 32);
        const uint32_t phase = (uint32_t)(it >> ITEM_BLOCK_BITS) & ((1u << ITEM_PHASE_BITS) - 1);
        const uint32_t item = (uint32_t)it & ((1u << ITEM_BLOCK_BITS) - 1);
        const hr_inst_dev I = load_uniform(insts[ii]);
        if (threadIdx.x == 0) {
            uint32_t go = 1;
            if (phase > 0) {
                const uint32_t* d = done + I.done_off + phase - 1;
                uint32_t spins = 0;
                while (__hip_atomic_load(d, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < I.items) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins >= spin_limit) {
                        go = 0;
                        hr_set_flag(base, HR_DEVF_STALL);
                        break;
                    }
                }
            }
            s_go = go;
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (uni(s_go)) {
            hr_env e = base;
            e.launch = phase & ((1u << hr::g::LAUNCH_BITS) - 1);
            e.launch_seq = phase;
            run_item(e, I, phase, item, smem);
        }
        __syncthreads();                                // every hook of the item is done
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(done + I.done_off + phase, 1u, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_item = claim(cursor, items, n_items);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_batch_wide(hr_env base, const hr_inst_dev* insts,
                                                     const uint64_t* items, uint32_t n_items,
                                                     uint32_t* cursor, uint32_t* done,
                                                     uint32_t spin_limit)
{
    batch_loop<4>(base, insts, items, n_items, cursor, done, spin_limit);
}

__global__ __launch_bounds__(1024, 8) void k_batch_dense(hr_env base, const hr_inst_dev* insts,
                                                         const uint64_t* items, uint32_t n_items,
                                                         uint32_t* cursor, uint32_t* done,
                                                         uint32_t spin_limit)
{
    batch_loop<8>(base, insts, items, n_items, cursor, done, spin_limit);
}

}  // namespace

bool hr_instance_shape(hr_instance& in, size_t elems[2], size_t* lds_bytes)
{
    // a job's phases are its launch epochs, which must stay distinct
    if (in.phases == 0 || in.phases > (1u << hr::g::LAUNCH_BITS)) return false;
    switch (in.pattern) {
    case HR_PAT_REDUCE: {
        const uint32_t n = in.n, T = in.threads;
        if (T == 0 || T > 1024 || T % 64 || in.blocks == 0 || in.phases != 1) return false;
        if (n < 2 || (n & (n - 1)) || n > 2 * T) return false;
        if (in.drop >= 31 - __builtin_clz(n)) return false;
        if (!in.data[0] || !in.data[1]) return false;
        elems[0] = (size_t)in.blocks * n;
        elems[1] = (size_t)in.blocks * T;
        *lds_bytes = (size_t)(HR_WORKER_THREADS / T) * n * 8;
        break;
    }
    case HR_PAT_JACOBI: {
        if (in.n == 0 || in.ny == 0 || !in.data[0] || !in.data[1]) return false;
        const uint64_t nbx = (in.n + 15) / 16, nby = (in.ny + 15) / 16;
        in.blocks = (uint32_t)(nbx * nby);
        in.threads = 256;
        elems[0] = elems[1] = (size_t)in.n * in.ny;
        *lds_bytes = (size_t)(HR_WORKER_THREADS / 256) * JACOBI_TILE_WORDS * 8;
        break;
    }
    case HR_PAT_LABELPROP: {
        const uint32_t T = in.threads;
        if (in.n == 0 || T == 0 || T > 1024 || T % 64) return false;
        if (!in.data[0] || !in.data[1] || !in.data[2] || !in.data[3]) return false;
        in.blocks = (in.n + T - 1) / T;
        elems[0] = in.n;
        elems[1] = 0;
        *lds_bytes = 0;
        break;
    }
    default:
        return false;
    }
    return in.blocks > 0 && in.blocks < (1u << ITEM_BLOCK_BITS);
}


hr_inst_dev hr_make_inst_dev(const hr_instance& in, const size_t elems[2], uint64_t* sh0,
                             uint64_t* sh1, uint32_t r0, uint32_t r1, uint32_t done_off)
{
    hr_inst_dev d{};
    d.pattern = in.pattern;
    d.blocks = in.blocks;
    d.threads = in.threads;
    d.phases = in.phases;
    d.n = in.n;
    d.ny = in.ny;
    d.nbx = (in.n + 15) / 16;
    d.drop = in.drop;
    d.done_off = done_off;
    d.lds_id = r0;
    d.pack = HR_WORKER_THREADS / in.threads;
    d.items = (in.blocks + d.pack - 1) / d.pack;
    d.lds_words = in.pattern == HR_PAT_REDUCE   ? 2 * in.n
                  : in.pattern == HR_PAT_JACOBI ? 2 * JACOBI_TILE_WORDS
                                                : 0;
    // row-major maps; a jacobi job's rows are nx elements wide
    const uint32_t cols = in.pattern == HR_PAT_JACOBI ? in.n : 0u;
    d.g0 = hr_gref{sh0, sh0 ? elems[0] : 0, r0, hr_lay_rows(cols)};
    d.g1 = hr_gref{sh1, sh1 ? elems[1] : 0, r1, hr_lay_rows(cols)};
    d.p0 = in.data[0];
    d.p1 = const_cast<void*>(in.data[1]);
    d.p2 = in.data[2];
    d.p3 = in.data[3];
    return d;
}

struct hr_batch_s {
    hr_ctx ctx;
    uint32_t n_inst;
    std::vector<hr_inst_dev> hd;          // host copy of the job table
    std::vector<uint32_t> rows;           // rows of each job's 2-D regions (jacobi), else 0
    uint32_t tile = 0;                    // shadow map of the jacobi jobs (hr_batch_tuning)
    uint32_t arena;                       // allocation holding every instance's shadow
    hr_inst_dev* d_inst = nullptr;
    uint64_t* d_items[2] = {nullptr, nullptr};   // phase-major, largest-first orders
    uint32_t n_items = 0;
    uint32_t* d_done = nullptr;
    uint32_t n_done = 0;
    uint32_t* d_cursor = nullptr;
    size_t lds_bytes = 0;
    uint32_t max_workers[2] = {0, 0};     // per kernel variant
};

extern "C" hr_status hr_batch_destroy(hr_batch b)
{
    if (!b) return HR_E_INVAL;
    hipError_t e = hipStreamSynchronize(b->ctx->stream);
    if (b->d_inst) (void)hipFree(b->d_inst);
    for (uint64_t* p : b->d_items)
        if (p) (void)hipFree(p);
    if (b->d_done) (void)hipFree(b->d_done);
    if (b->d_cursor) (void)hipFree(b->d_cursor);
    if (b->arena != UINT32_MAX) hr_free_alloc(b->ctx, b->arena);
    delete b;
    return e == hipSuccess ? HR_OK : HR_E_HIP;
}

extern "C" hr_status hr_batch_create(hr_ctx c, hr_instance* inst, uint32_t n_inst, hr_batch* out)
{
    if (!c || !inst || !out || n_inst == 0 || n_inst >= (1u << 24)) return HR_E_INVAL;
    *out = nullptr;
    if (c->cfg.flags & (HR_CFG_WORD4 | HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE))
        return HR_E_INVAL;   // the arena holds flat 8-byte words
    std::vector<size_t> el(2 * (size_t)n_inst), words(2 * (size_t)n_inst);
    size_t total = 0, lds = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        size_t lb = 0;
        if (!hr_instance_shape(inst[i], &el[2 * i], &lb)) return HR_E_INVAL;
        for (int k = 0; k < 2; ++k) words[2 * i + k] = el[2 * i + k];
        if (inst[i].pattern == HR_PAT_JACOBI) {
            // room for every tiled shadow map: both sides padded to whole
            // tiles of the largest side
            constexpr size_t T = size_t(1) << HR_TILE_LOG2_MAX;
            const size_t padded = ((inst[i].ny + T - 1) / T * T) * ((inst[i].n + T - 1) / T * T);
            words[2 * i] = words[2 * i + 1] = padded;
        }
        total += words[2 * i] + words[2 * i + 1];
        lds = std::max(lds, lb);
    }
    hr_batch b = new (std::nothrow) hr_batch_s();
    if (!b) return HR_E_NOMEM;
    b->ctx = c;
    b->n_inst = n_inst;
    b->arena = UINT32_MAX;
    b->lds_bytes = lds;
    uint32_t arena = 0;
    hr_status st = hr_new_alloc(c, total, &arena);
    if (st != HR_OK) {
        delete b;
        return st;
    }
    b->arena = arena;
    std::vector<hr_inst_dev>& hd = b->hd;
    hd.resize(n_inst);
    b->rows.assign(n_inst, 0u);
    uint64_t* base = c->allocs[arena].mem;
    size_t off = 0;
    uint32_t done_off = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        hr_instance& in = inst[i];
        in.region[0] = in.region[1] = UINT32_MAX;
        if (in.pattern == HR_PAT_JACOBI) b->rows[i] = in.ny;
        uint64_t* sh[2] = {nullptr, nullptr};
        for (int k = 0; k < 2; ++k) {
            if (!el[2 * i + k]) continue;
            sh[k] = base + off;
            in.region[k] = hr_new_region(c, in.data[k], el[2 * i + k], sh[k], arena);
            off += words[2 * i + k];
        }
        hd[i] = hr_make_inst_dev(in, &el[2 * i], sh[0], sh[1], in.region[0], in.region[1],
                                 done_off);
        done_off += in.phases;
    }
    b->n_done = done_off;
    // Work queues.  Order 0: phase-major, instances in given order.  Order
    // 1: phase-major, instances with the most blocks first in every phase.
    std::vector<uint32_t> by_size(n_inst);
    std::iota(by_size.begin(), by_size.end(), 0u);
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](uint32_t x, uint32_t y) { return inst[x].blocks > inst[y].blocks; });
    uint32_t max_phase = 0;
    for (uint32_t i = 0; i < n_inst; ++i) max_phase = std::max(max_phase, inst[i].phases);
    std::vector<uint64_t> q[2];
    for (int o = 0; o < 2; ++o) {
        for (uint32_t p = 0; p < max_phase; ++p)
            for (uint32_t k = 0; k < n_inst; ++k) {
                const uint32_t i = o ? by_size[k] : k;
                if (p >= inst[i].phases) continue;
                for (uint32_t it = 0; it < hd[i].items; ++it)
                    q[o].push_back(((uint64_t)i << 32) | ((uint64_t)p << ITEM_BLOCK_BITS) | it);
            }
    }
    b->n_items = (uint32_t)q[0].size();
    if (q[0].size() >= (1ull << 32)) {
        hr_batch_destroy(b);
        return HR_E_INVAL;
    }
    if (hipMalloc(&b->d_inst, sizeof(hr_inst_dev) * n_inst) != hipSuccess ||
        hipMalloc(&b->d_items[0], sizeof(uint64_t) * q[0].size()) != hipSuccess ||
        hipMalloc(&b->d_items[1], sizeof(uint64_t) * q[1].size()) != hipSuccess ||
        hipMalloc(&b->d_done, sizeof(uint32_t) * b->n_done) != hipSuccess ||
        hipMalloc(&b->d_cursor, sizeof(uint32_t)) != hipSuccess) {
        hr_batch_destroy(b);
        return HR_E_NOMEM;
    }
    if (hipMemcpy(b->d_inst, hd.data(), sizeof(hr_inst_dev) * n_inst, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(b->d_items[0], q[0].data(), sizeof(uint64_t) * q[0].size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_items[1], q[1].data(), sizeof(uint64_t) * q[1].size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
        hr_batch_destroy(b);
        return HR_E_HIP;
    }
    int per_cu[2] = {0, 0}, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[0], k_batch_wide, 1024,
                                                     b->lds_bytes) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[1], k_batch_dense, 1024,
                                                     b->lds_bytes) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess ||
        per_cu[0] <= 0 || per_cu[1] <= 0 || cus <= 0) {
        hr_batch_destroy(b);
        return HR_E_HIP;
    }
    b->max_workers[0] = (uint32_t)(per_cu[0] * cus);
    b->max_workers[1] = (uint32_t)(per_cu[1] * cus);
    *out = b;
    return HR_OK;
}

extern "C" hr_status hr_batch_info(hr_batch b, uint32_t variant, uint32_t* max_workers,
                                   uint64_t* items)
{
    if (!b || variant > 1) return HR_E_INVAL;
    if (max_workers) *max_workers = b->max_workers[variant];
    if (items) *items = b->n_items;
    return HR_OK;
}

extern "C" hr_status hr_batch_run(hr_batch b, const hr_batch_tuning* tune, void* stream)
{
    if (!b) return HR_E_INVAL;
    hr_batch_tuning t = {};
    if (tune) t = *tune;
    if (t.order > 1 || t.variant > 1) return HR_E_INVAL;
    if (t.coalesce > 1 && !hr_coalesce_width_ok(t.coalesce)) return HR_E_INVAL;
    const uint32_t cap = b->max_workers[t.variant];
    const uint32_t workers = t.workers ? std::min(t.workers, cap) : cap;
    const uint32_t spin = t.spin_limit ? t.spin_limit : (1u << 24);
    const uint32_t tw = t.tile & 15u, th = (t.tile >> 4) & 15u;
    if ((t.tile >> 8) || tw > HR_TILE_LOG2_MAX || th > HR_TILE_LOG2_MAX) return HR_E_INVAL;
    hr_ctx c = b->ctx;
    hipStream_t s = hr_stream(c, stream);
    if (t.tile != b->tile) {
        // Another shadow map for the jacobi jobs: their descriptors and
        // regions take it (the arena has room for the padding), once the
        // runs before that read the old table have finished.
        for (uint32_t i = 0; i < b->n_inst; ++i) {
            if (!b->rows[i]) continue;
            hr_inst_dev& d = b->hd[i];
            const uint32_t nx = d.n;
            const hr_lay tiled{nx, (nx + (1u << tw) - 1u) >> tw, tw, th};
            d.g0.lay = d.g1.lay = t.tile ? tiled : hr_lay_rows(nx);
            for (uint32_t r : {d.g0.id, d.g1.id}) {
                c->reg[r].lay = t.tile ? tiled : hr_lay{};
                c->reg[r].rows = b->rows[i];
            }
        }
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(b->d_inst, b->hd.data(), sizeof(hr_inst_dev) * b->n_inst,
                      hipMemcpyHostToDevice) != hipSuccess)
            return HR_E_HIP;
        b->tile = t.tile;
    }
    // every run starts from initial shadow and empty phase counters
    if (hr_fill64(c->allocs[b->arena].mem, c->allocs[b->arena].words, s) != hipSuccess ||
        hr_fill32(b->d_done, b->n_done, s) != hipSuccess ||
        hr_fill32(b->d_cursor, 1, s) != hipSuccess)
        return HR_E_HIP;
    hr_env e = hr_make_env(c);
    e.site_limit = 0;   // site ids are per job; the limit does not apply to a batch
    if (t.coalesce) e.group = t.coalesce == 1 ? 0u : t.coalesce;
    if (t.variant == 0)
        HR_LAUNCH(k_batch_wide, dim3(workers), dim3(1024), b->lds_bytes, s, e, b->d_inst,
                  b->d_items[t.order], b->n_items, b->d_cursor, b->d_done, spin);
    else
        HR_LAUNCH(k_batch_dense, dim3(workers), dim3(1024), b->lds_bytes, s, e, b->d_inst,
                  b->d_items[t.order], b->n_items, b->d_cursor, b->d_done, spin);
    return HR_OK;
}

// ----------------------------------------------------------------------
// The serial path: one job at a time with its own context and shadow.
extern "C" hr_status hr_job_run(const hr_instance* inst, const hr_config* cfg, hr_race* out,
                                size_t cap, size_t* n_out, void* stream)
{
    if (!inst || !n_out) return HR_E_INVAL;
    hr_instance in = *inst;
    size_t el[2] = {0, 0}, lds = 0;
    if (!hr_instance_shape(in, el, &lds)) return HR_E_INVAL;
    hr_ctx c = nullptr;
    hr_status st = hr_ctx_create(&c, cfg, stream);
    if (st != HR_OK) return st;
    uint32_t r[2] = {UINT32_MAX, UINT32_MAX};
    for (int k = 0; k < 2 && st == HR_OK; ++k)
        if (el[k]) st = hr_shadow_alloc(c, in.data[k], el[k] * 4, 4, &r[k]);
    for (uint32_t p = 0; p < in.phases && st == HR_OK; ++p) {
        switch (in.pattern) {
        case HR_PAT_REDUCE:
            st = hr_reduce_check(c, r[0], r[1], (const int32_t*)in.data[0], (int32_t*)in.data[1],
                                 in.n, in.threads, in.blocks, in.drop, stream);
            break;
        case HR_PAT_JACOBI: {
            const int o = p & 1;
            st = hr_jacobi_check(c, r[o], r[1 - o], (const float*)in.data[o],
                                 (float*)const_cast<void*>(in.data[1 - o]), in.ny, in.n,
                                 (const int32_t*)in.data[2], stream);
            break;
        }
        default:
            st = hr_labelprop_check(c, r[0], UINT32_MAX, UINT32_MAX,
                                    (int32_t*)const_cast<void*>(in.data[0]),
                                    (const int32_t*)in.data[1], (const int32_t*)in.data[2],
                                    (const uint8_t*)in.data[3], in.n, in.threads, stream);
            break;
        }
        if (st == HR_OK) st = hr_kernel_end(c, stream);
    }
    hr_status rep = st;
    if (st == HR_OK) rep = hr_report(c, out, cap, n_out, stream);
    const hr_status ds = hr_ctx_destroy(c);
    if (rep != HR_OK) return rep;
    return ds;
}
