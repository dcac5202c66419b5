// Serving: a stream of check jobs with continuous batching at the
// granularity of one phase (one launch of a job's kernel).
//
// The host loop admits jobs that have arrived, in arrival order, while a
// job slot and shadow memory under the budget are free; every iteration is
// one launch with one 1024-thread block per work item of every resident
// job's next phase, so jobs that arrive while others run join at the next
// iteration and their work shares the device with everyone else's.  The launch boundary of every iteration
// is the launch boundary of each job's phase; a job's shadow stays resident
// across its phases (its launch epoch is its phase) and is released when its
// last phase is reported.  No kernel waits for another block: items of one
// iteration are independent.
//
// The serial path replays the same arrivals one job at a time through
// hr_job_run (own context, shadow allocation, one launch per phase, report,
// free).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <thread>
#include <vector>

#include "hr.h"
#include "hr_arena.h"
#include "hr_exec.h"
#include "hr_internal.h"

namespace {

// One iteration: work item blockIdx.x of the flat list of the resident
// jobs' items, each job contributing the items of its next phase (prefix[k]
// = items of the jobs before job k in the list).
// PATTERNS: the workload patterns the iteration's jobs may have (run_item).
template <uint32_t PATTERNS>
__global__ __launch_bounds__(1024, 8) void k_iter(hr_env base, const hr_inst_dev* __restrict__ slots,
                                               const uint32_t* __restrict__ act,
                                               const uint64_t* __restrict__ prefix, uint32_t n_act)
{
    extern __shared__ uint32_t smem[];
    const uint32_t i = blockIdx.x;
    // the job owning item i: the largest k with prefix[k] <= i
    uint32_t lo = 0, hi = n_act;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (uni64(prefix[mid]) <= i) lo = mid;
        else hi = mid;
    }
    const uint32_t a = uni(act[lo]);
    const uint32_t slot = a & 0xFFFFFu, phase = a >> 20;
    const uint32_t item = i - (uint32_t)uni64(prefix[lo]);
    const hr_inst_dev I = load_uniform(slots[slot]);
    hr_env e = base;
    e.launch = phase & ((1u << hr::g::LAUNCH_BITS) - 1);
    e.launch_seq = phase;
    run_item<PATTERNS>(e, I, phase, item, smem);
}

// One phase of a stencil job of the large lane: the stencil's tuned body,
// four tiles to a 1024-thread block (k_jacobi_x4), on the job's shadow
// words in the arena, under the lane's environment with the phase's launch
// epoch.
hr_status launch_stencil_phase(const hr_env& e, const hr_inst_dev& d, uint32_t phase,
                               hipStream_t s)
{
    const bool odd = phase & 1u;
    hr_kargs a{};
    a.env = e;
    a.env.launch = phase & ((1u << hr::g::LAUNCH_BITS) - 1);
    a.env.launch_seq = phase;
    const uint32_t nbx = (d.n + 15) / 16, tiles = nbx * ((d.ny + 15) / 16);
    HR_LAUNCH(k_jacobi_x4<1>, dim3((tiles + 3) / 4), dim3(1024), 0, s, a, odd ? d.g1 : d.g0,
              odd ? d.g0 : d.g1, (const float*)(odd ? d.p1 : d.p0), (float*)(odd ? d.p0 : d.p1),
              d.ny, d.n, nbx, tiles, (const int32_t*)d.p2);
    return HR_OK;
}

using iter_kernel = void (*)(hr_env, const hr_inst_dev*, const uint32_t*, const uint64_t*,
                             uint32_t);

// The iteration kernel for a set of patterns (bit p: pattern p): one built
// for that pattern alone when there is one, else the one for all.
iter_kernel iter_for(uint32_t patterns)
{
    switch (patterns) {
    case 1u << HR_PAT_REDUCE: return k_iter<1u << HR_PAT_REDUCE>;
    case 1u << HR_PAT_JACOBI: return k_iter<1u << HR_PAT_JACOBI>;
    case 1u << HR_PAT_LABELPROP: return k_iter<1u << HR_PAT_LABELPROP>;
    default: return k_iter<HR_ALL_PATTERNS>;
    }
}

constexpr uint64_t GRANULE_WORDS = 32;   // 256 bytes of 8-byte shadow words

struct job_state {
    hr_instance in;
    size_t elems[2] = {0, 0};
    uint64_t off = 0, granules = 0;   // arena placement
    uint32_t items = 0;               // work items of one phase
    uint32_t slot = 0, phase = 0;
    uint32_t burst = 1;               // phases its lane's iteration in flight runs
    int32_t status = 0;
    bool running = false;             // in its lane's iteration in flight
};

using clock_t_ = std::chrono::steady_clock;

double seconds_since(clock_t_::time_point t0)
{
    return std::chrono::duration<double>(clock_t_::now() - t0).count();
}

void wait_until(clock_t_::time_point t0, double at)
{
    for (;;) {
        const double left = at - seconds_since(t0);
        if (left <= 0) return;
        if (left > 2e-3) std::this_thread::sleep_for(std::chrono::microseconds((int64_t)(left * 5e5)));
        else std::this_thread::yield();
    }
}

hr_race tag_region(hr_race r, uint32_t job)
{
    r.region = 2u * job + (r.space == HR_LDS ? 0u : std::min(r.region, 1u));
    return r;
}

hr_status serve_serial(hr_ctx c, const hr_instance* jobs, hr_serve_job* times, uint32_t n,
                       std::vector<hr_race>& all, void* stream)
{
    const auto t0 = clock_t_::now();
    std::vector<hr_race> buf(4096);
    for (uint32_t j = 0; j < n; ++j) {
        wait_until(t0, times[j].arrival_s);
        times[j].admit_s = seconds_since(t0);
        size_t got = 0;
        hr_status st;
        for (;;) {
            st = hr_job_run(&jobs[j], &c->cfg, buf.data(), buf.size(), &got, stream);
            if (st == HR_E_INVAL && got > buf.size()) {
                buf.resize(got);
                continue;
            }
            break;
        }
        times[j].finish_s = seconds_since(t0);
        times[j].status = st;
        if (st < 0) return st;
        for (size_t i = 0; i < got; ++i) all.push_back(tag_region(buf[i], j));
    }
    return HR_OK;
}

// Jobs run in lanes by class: a lane has its own stream, ring and counters
// and runs its iterations one after another, while the lanes' iterations
// overlap on the device.  An iteration lasts as long as its slowest item,
// so jobs whose phases are long (label propagation, bound by the edge list
// of its largest hub, which grows with the graph; jobs of many items) would
// hold back the short jobs sharing their iterations.  Four lanes: as many as
// the device's hardware queues for one process.
//
// The short-job lane runs two phases of its jobs per iteration
// (hr_serve_config.lane_burst), as two launches back to back: a small
// stencil's 20 phases then cost 10 host round trips instead of 20, while a
// job that arrives meanwhile waits for at most two launches.
//
// The large lane runs its jobs one at a time, in admission order: a job of
// that many items fills the device by itself, so sharing iterations among
// several would only stretch every one of them (each would finish near the
// end of their common span), and one job at a time keeps the blocks in
// flight to one job's grid, leaving room for the short lanes as they
// retire.  A stencil job there runs all its remaining phases in one
// iteration, as back-to-back launches of the tuned stencil body (the one a
// standalone check runs, four tiles to a 1024-thread block so that the
// short lanes' blocks find room beside it), each phase with its own launch
// epoch; hr_serve_config.large_burst caps the phases of one iteration.
constexpr uint32_t N_LANES = 4;
constexpr uint32_t LANE_SHORT = 0, LANE_GRAPH = 1, LANE_LARGE = 2, LANE_LARGE_GRAPH = 3;
constexpr uint32_t LARGE_ITEMS = 1024;        // items per phase above which a job is large
constexpr uint32_t LARGE_GRAPH_ITEMS = 64;    // the same for label propagation (64 K vertices)

uint32_t lane_of(const hr_instance& in, uint32_t items)
{
    if (in.pattern == HR_PAT_LABELPROP)
        return items >= LARGE_GRAPH_ITEMS ? LANE_LARGE_GRAPH : LANE_GRAPH;
    return items > LARGE_ITEMS ? LANE_LARGE : LANE_SHORT;
}

struct lane_state {
    hipStream_t s = nullptr;
    bool own_stream = false;
    hipEvent_t done = nullptr;
    hr_race_rec* ring = nullptr;     // the context's ring and counters for the
    uint32_t* ctr = nullptr;         // first lane, own ones for the others
    bool own_ring = false;
    uint32_t* act = nullptr;         // device copies of the job lists of the
    uint64_t* prefix = nullptr;      // iterations one burst launches (max_slots each)
    uint32_t* h_act = nullptr;       // pinned staging
    uint64_t* h_prefix = nullptr;
    uint32_t* h_ctr = nullptr;       // counters after the iteration
    size_t lds = 0;                  // dynamic LDS of the lane's iterations
    std::vector<uint32_t> jobs;      // resident jobs of the lane, in admission order
    bool in_flight = false;
};

struct serve_buffers {
    uint64_t* arena = nullptr;
    hr_inst_dev* slots = nullptr;
    hr_inst_dev* h_desc = nullptr;   // pinned staging
    lane_state lane[N_LANES];
    ~serve_buffers()
    {
        for (lane_state& L : lane)
            if (L.s) (void)hipStreamSynchronize(L.s);   // nothing in flight uses what is freed
        for (lane_state& L : lane) {
            if (L.own_stream && L.s) (void)hipStreamDestroy(L.s);
            if (L.done) (void)hipEventDestroy(L.done);
            if (L.own_ring) {
                if (L.ring) (void)hipFree(L.ring);
                if (L.ctr) (void)hipFree(L.ctr);
            }
            if (L.act) (void)hipFree(L.act);
            if (L.prefix) (void)hipFree(L.prefix);
            if (L.h_act) (void)hipHostFree(L.h_act);
            if (L.h_prefix) (void)hipHostFree(L.h_prefix);
            if (L.h_ctr) (void)hipHostFree(L.h_ctr);
        }
        if (arena) (void)hipFree(arena);
        if (slots) (void)hipFree(slots);
        if (h_desc) (void)hipHostFree(h_desc);
    }
};

// burst: iterations a lane enqueues at once (each with its own job list).
hr_status lane_init(lane_state& L, hr_ctx c, hipStream_t caller, bool first, uint32_t max_slots,
                    uint32_t burst)
{
    if (first) {
        L.s = caller;
        L.ring = c->ring;
        L.ctr = c->ctr;
    } else {
        if (hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) != hipSuccess) return HR_E_HIP;
        L.own_stream = true;
        L.own_ring = true;
        if (hipMalloc(&L.ring, sizeof(hr_race_rec) * std::max(1u, c->cfg.ring_capacity)) !=
                hipSuccess ||
            hipMalloc(&L.ctr, sizeof(uint32_t) * HR_CTR_WORDS) != hipSuccess)
            return HR_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) return HR_E_HIP;
    const size_t na = (size_t)max_slots * burst, np = (size_t)(max_slots + 1) * burst;
    if (hipMalloc(&L.act, sizeof(uint32_t) * na) != hipSuccess ||
        hipMalloc(&L.prefix, sizeof(uint64_t) * np) != hipSuccess ||
        hipHostMalloc(&L.h_act, sizeof(uint32_t) * na, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&L.h_prefix, sizeof(uint64_t) * np, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&L.h_ctr, sizeof(uint32_t) * HR_CTR_SITES, hipHostMallocDefault) !=
            hipSuccess)
        return HR_E_NOMEM;
    return HR_OK;
}

hr_status serve_continuous(hr_ctx c, const hr_instance* jobs, hr_serve_job* times, uint32_t n,
                           const hr_serve_config& cfg, std::vector<hr_race>& all, void* stream)
{
    std::vector<job_state> js(n);
    std::vector<uint32_t> lane_of_job(n);
    size_t lds[N_LANES] = {};
    const uint64_t budget_granules = cfg.shadow_budget / (GRANULE_WORDS * 8);
    uint64_t need = 0;
    for (uint32_t j = 0; j < n; ++j) {
        js[j].in = jobs[j];
        size_t l = 0;
        if (!hr_instance_shape(js[j].in, js[j].elems, &l)) return HR_E_INVAL;
        const uint64_t words = js[j].elems[0] + js[j].elems[1];
        js[j].granules = (words + GRANULE_WORDS - 1) / GRANULE_WORDS + 1;
        if (js[j].granules > budget_granules) return HR_E_NOMEM;   // could never be admitted
        js[j].items = hr_make_inst_dev(js[j].in, js[j].elems, nullptr, nullptr, 0, 0, 0).items;
        if (js[j].items > cfg.max_items) return HR_E_INVAL;         // nor this one
        lane_of_job[j] = lane_of(js[j].in, js[j].items);
        lds[lane_of_job[j]] = std::max(lds[lane_of_job[j]], l);
        need += js[j].granules;
    }
    // the arena never needs more than every job at once
    const uint64_t arena_granules = std::min(budget_granules, need);
    const uint32_t max_slots = cfg.max_slots;
    serve_buffers b;
    if (hipMalloc(&b.arena, arena_granules * GRANULE_WORDS * 8) != hipSuccess ||
        hipMalloc(&b.slots, sizeof(hr_inst_dev) * max_slots) != hipSuccess ||
        hipHostMalloc(&b.h_desc, sizeof(hr_inst_dev) * max_slots, hipHostMallocDefault) !=
            hipSuccess)
        return HR_E_NOMEM;
    hr_env env[N_LANES];
    const hr_env env_base = hr_make_env(c);
    for (uint32_t k = 0; k < N_LANES; ++k) {
        lane_state& L = b.lane[k];
        const hr_status st = lane_init(L, c, hr_stream(c, stream), k == 0, max_slots,
                                       k == LANE_SHORT ? cfg.lane_burst : 1u);
        if (st != HR_OK) return st;
        L.lds = lds[k];
        for (uint32_t pm : {1u << HR_PAT_REDUCE, 1u << HR_PAT_JACOBI, 1u << HR_PAT_LABELPROP,
                            HR_ALL_PATTERNS}) {
            int per_cu = 0;   // the iteration kernels must fit with the lane's largest LDS
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, iter_for(pm),
                                                             HR_WORKER_THREADS, L.lds) !=
                    hipSuccess ||
                per_cu <= 0)
                return HR_E_HIP;
        }
        env[k] = env_base;
        env[k].ring = L.ring;
        env[k].ctr = L.ctr;
        env[k].site_limit = 0;   // site ids are per job; the limit does not apply here
        env[k].log = nullptr;    // nor does the access log: lane counters restart per iteration
    }
    arena_alloc arena(arena_granules);
    std::vector<uint32_t> free_slots;
    for (uint32_t k = max_slots; k-- > 0;) free_slots.push_back(k);
    std::vector<hr_race> ring(c->cfg.ring_capacity);
    uint32_t next = 0, finished = 0;
    uint64_t resident_items = 0;   // items of one phase of every resident job
    const auto t0 = clock_t_::now();
    while (finished < n) {
        // admit arrived jobs in order while a slot, shadow memory and room
        // under the item cap are free; a job joins its lane's next iteration
        const double now = seconds_since(t0);
        while (next < n && times[next].arrival_s <= now && !free_slots.empty()) {
            job_state& st = js[next];
            if (resident_items + st.items > cfg.max_items) break;
            uint64_t off = 0;
            if (!arena.alloc(st.granules, &off)) break;
            resident_items += st.items;
            st.off = off;
            st.slot = free_slots.back();
            free_slots.pop_back();
            lane_state& L = b.lane[lane_of_job[next]];
            uint64_t* sh0 = b.arena + off * GRANULE_WORDS;
            uint64_t* sh1 = st.elems[1] ? sh0 + st.elems[0] : nullptr;
            if (hr_fill64(sh0, st.elems[0] + st.elems[1], L.s) != hipSuccess) return HR_E_HIP;
            b.h_desc[st.slot] = hr_make_inst_dev(st.in, st.elems, sh0, sh1, 2 * next, 2 * next + 1, 0);
            if (hipMemcpyAsync(b.slots + st.slot, b.h_desc + st.slot, sizeof(hr_inst_dev),
                               hipMemcpyHostToDevice, L.s) != hipSuccess)
                return HR_E_HIP;
            times[next].admit_s = now;
            L.jobs.push_back(next);
            ++next;
        }
        // an idle lane with resident jobs starts its next iteration: the next
        // phase of each of them (the large lane: of its first job)
        for (uint32_t k = 0; k < N_LANES; ++k) {
            lane_state& L = b.lane[k];
            if (L.in_flight || L.jobs.empty()) continue;
            const size_t n_run = k == LANE_LARGE ? 1 : L.jobs.size();
            if (hr_fill32(L.ctr, HR_CTR_WORDS, L.s) != hipSuccess) return HR_E_HIP;
            job_state& first = js[L.jobs[0]];
            if (k == LANE_LARGE && first.in.pattern == HR_PAT_JACOBI) {
                // its next phases, one launch of the stencil kernel each
                const hr_inst_dev& d = b.h_desc[first.slot];
                const uint32_t last = cfg.large_burst
                                          ? std::min(first.in.phases, first.phase + cfg.large_burst)
                                          : first.in.phases;
                for (uint32_t p = first.phase; p < last; ++p) {
                    const hr_status ls = launch_stencil_phase(env[k], d, p, L.s);
                    if (ls != HR_OK) return ls;
                }
                first.burst = last - first.phase;
            } else {
                // iteration j of the burst runs phase phase + j of every job
                // that has it; each iteration has its own job list
                const uint32_t burst = k == LANE_SHORT ? cfg.lane_burst : 1u;
                uint32_t iters = 0;
                for (uint32_t j = 0; j < burst; ++j) {
                    uint32_t* act = L.h_act + (size_t)j * max_slots;
                    uint64_t* pre = L.h_prefix + (size_t)j * (max_slots + 1);
                    uint64_t total = 0;
                    uint32_t patterns = 0, m = 0;
                    for (size_t q = 0; q < n_run; ++q) {
                        const job_state& st = js[L.jobs[q]];
                        if (st.phase + j >= st.in.phases) continue;
                        pre[m] = total;
                        act[m] = st.slot | ((st.phase + j) << 20);
                        total += st.items;
                        patterns |= 1u << st.in.pattern;
                        ++m;
                    }
                    if (m == 0) break;
                    pre[m] = total;
                    uint32_t* d_act = L.act + (size_t)j * max_slots;
                    uint64_t* d_pre = L.prefix + (size_t)j * (max_slots + 1);
                    if (hipMemcpyAsync(d_act, act, sizeof(uint32_t) * m, hipMemcpyHostToDevice,
                                       L.s) != hipSuccess ||
                        hipMemcpyAsync(d_pre, pre, sizeof(uint64_t) * (m + 1),
                                       hipMemcpyHostToDevice, L.s) != hipSuccess)
                        return HR_E_HIP;
                    HR_LAUNCH(iter_for(patterns), dim3((uint32_t)total), dim3(HR_WORKER_THREADS),
                              L.lds, L.s, env[k], b.slots, d_act, d_pre, m);
                    ++iters;
                }
                for (size_t q = 0; q < n_run; ++q) {
                    job_state& st = js[L.jobs[q]];
                    st.burst = std::min(iters, st.in.phases - st.phase);
                }
            }
            if (hipMemcpyAsync(L.h_ctr, L.ctr, sizeof(uint32_t) * HR_CTR_SITES,
                               hipMemcpyDeviceToHost, L.s) != hipSuccess ||
                hipEventRecord(L.done, L.s) != hipSuccess)
                return HR_E_HIP;
            for (size_t q = 0; q < n_run; ++q) js[L.jobs[q]].running = true;
            L.in_flight = true;
        }
        // collect the lanes whose iteration has finished
        bool progressed = false;
        for (uint32_t k = 0; k < N_LANES; ++k) {
            lane_state& L = b.lane[k];
            if (!L.in_flight) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return HR_E_HIP;
            L.in_flight = false;
            progressed = true;
            const uint32_t head = L.h_ctr[HR_CTR_HEAD], flags = L.h_ctr[HR_CTR_FLAGS];
            const uint32_t got = std::min(head, c->cfg.ring_capacity);
            if (got && (hipMemcpyAsync(ring.data(), L.ring, sizeof(hr_race_rec) * got,
                                       hipMemcpyDeviceToHost, L.s) != hipSuccess ||
                        hipStreamSynchronize(L.s) != hipSuccess))
                return HR_E_HIP;
            // the descriptors carry 2*job (+1) as report ids
            all.insert(all.end(), ring.begin(), ring.begin() + got);
            int warn = 0;
            if (flags & HR_DEVF_CLOCK) warn |= HR_W_CLOCK_OVERFLOW;
            if (flags & HR_DEVF_RANGE) warn |= HR_W_OUT_OF_RANGE;
            if (flags & HR_DEVF_STALL) warn |= HR_W_STALLED;
            if (head > c->cfg.ring_capacity) {
                // recover the global part of the iteration's jobs from their
                // sticky race words
                warn |= HR_W_RING_OVERFLOW;
                for (uint32_t j : L.jobs) {
                    const job_state& st = js[j];
                    if (!st.running) continue;
                    std::vector<uint64_t> sh(st.elems[0] + st.elems[1]);
                    if (hipMemcpyAsync(sh.data(), b.arena + st.off * GRANULE_WORDS, 8 * sh.size(),
                                       hipMemcpyDeviceToHost, L.s) != hipSuccess ||
                        hipStreamSynchronize(L.s) != hipSuccess)
                        return HR_E_HIP;
                    for (size_t i = 0; i < sh.size(); ++i) {
                        if ((sh[i] & hr::g::TAG_M) != hr::T_RACE) continue;
                        hr_race r = {};
                        r.space = HR_GLOBAL;
                        r.region = 2 * j + (i >= st.elems[0] ? 1 : 0);
                        r.index = i >= st.elems[0] ? i - st.elems[0] : i;
                        r.block = r.launch = r.tid = 0xFFFFFFFFu;
                        r.flags = HR_RACE_SCANNED;
                        all.push_back(r);
                    }
                }
            }
            // advance, and retire the jobs whose last phase just ran; jobs
            // admitted during the iteration keep their place
            const double end = seconds_since(t0);
            std::vector<uint32_t> still;
            for (uint32_t j : L.jobs) {
                job_state& st = js[j];
                if (!st.running) {
                    still.push_back(j);
                    continue;
                }
                st.running = false;
                st.status |= warn;
                st.phase += st.burst;
                if (st.phase < st.in.phases) {
                    still.push_back(j);
                    continue;
                }
                times[j].finish_s = end;
                times[j].status = st.status;
                resident_items -= st.items;
                arena.release(st.off, st.granules);
                free_slots.push_back(st.slot);
                ++finished;
            }
            L.jobs.swap(still);
        }
        if (progressed || finished == n) continue;
        bool busy = false;
        for (const lane_state& L : b.lane) busy |= L.in_flight;
        if (!busy && next < n) {
            wait_until(t0, times[next].arrival_s);   // nothing resident: wait for the next job
        } else if (busy) {
            // wait for an iteration or the next arrival, whichever comes first
            const double until = next < n ? times[next].arrival_s : 1e300;
            const double left = until - seconds_since(t0);
            if (left > 0) std::this_thread::sleep_for(std::chrono::microseconds(
                              std::max<int64_t>(1, std::min<int64_t>(20, (int64_t)(left * 1e6)))));
        }
    }
    return HR_OK;
}

bool race_key_less(const hr_race& a, const hr_race& b)
{
    const uint32_t ka = a.space == HR_LDS ? a.block : 0u, kb = b.space == HR_LDS ? b.block : 0u;
    if (a.region != b.region) return a.region < b.region;
    if (a.space != b.space) return a.space < b.space;
    if (ka != kb) return ka < kb;
    return a.index < b.index;
}

bool race_key_same(const hr_race& a, const hr_race& b)
{
    return a.region == b.region && a.space == b.space && a.index == b.index &&
           (a.space != HR_LDS || a.block == b.block);
}

}  // namespace

extern "C" hr_status hr_serve(hr_ctx c, const hr_instance* jobs, hr_serve_job* times,
                              uint32_t n_jobs, const hr_serve_config* cfg_in, hr_race* out,
                              size_t cap, size_t* n_out, void* stream)
{
    if (!c || !jobs || !times || !n_out || n_jobs == 0 || n_jobs >= (1u << 30)) return HR_E_INVAL;
    if (c->cfg.flags & (HR_CFG_WORD4 | HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE))
        return HR_E_INVAL;   // the arenas hold flat 8-byte words
    hr_serve_config cfg = {};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.max_slots == 0) cfg.max_slots = 1024;
    if (cfg.shadow_budget == 0) cfg.shadow_budget = 64ull << 30;
    if (cfg.max_items == 0) cfg.max_items = HR_SERVE_MAX_ITEMS;
    if (cfg.lane_burst == 0) cfg.lane_burst = 2;
    if (cfg.max_slots >= (1u << 20) || cfg.max_items > HR_SERVE_MAX_ITEMS ||
        cfg.lane_burst > 64)
        return HR_E_INVAL;
    for (uint32_t j = 0; j < n_jobs; ++j) {
        times[j].admit_s = times[j].finish_s = -1.0;
        times[j].flagged = 0;
        times[j].status = 0;
        if (j && times[j].arrival_s < times[j - 1].arrival_s) return HR_E_INVAL;
    }
    std::vector<hr_race> all;
    const hr_status st = cfg.serial ? serve_serial(c, jobs, times, n_jobs, all, stream)
                                    : serve_continuous(c, jobs, times, n_jobs, cfg, all, stream);
    if (st < 0) return st;
    std::sort(all.begin(), all.end(), race_key_less);
    size_t n = 0;
    for (size_t i = 0; i < all.size(); ++i)
        if (n == 0 || !race_key_same(all[n - 1], all[i])) all[n++] = all[i];
    for (size_t i = 0; i < n; ++i) times[all[i].region / 2].flagged += 1;
    *n_out = n;
    if (n > cap || (n && !out)) return HR_E_INVAL;
    std::copy(all.begin(), all.begin() + n, out);
    return HR_OK;
}
