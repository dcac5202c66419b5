// Device side of the race checker: what instrumented HIP kernels call.
//
//   hr_thread t = hr_thread_make(args.env, logical_block, thread_in_block);
//   ... data access ...;  hr_access<HR_READ>(args, t, region, index);
//   hr_barrier_block(args.env, t);   // replaces __syncthreads()
//   hr_barrier_wave(args.env, t);    // wave-scope barrier
//
// Each hook is the lock-free shadow update of the paper's Algorithm 1
// (Sec. IV-B): read the shadow word, derive the thread relation and sync
// status, step the state machine, and publish the new word atomically.  The
// hook need not be atomic with the access it checks (Sec. III-A, Scenario 1);
// it only has to finish before the thread passes its next barrier or its
// launch ends.  Every hook has the result of its own atomics before then (a
// hook split in two, issue and settle, reads it at the settle, still before
// the barrier), so shadow updates are applied in an order consistent with
// happens-before.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr.h"
#include "hr_fsm.h"

#define HR_MAX_REGIONS 16   // regions addressable by kernel arguments

// Device-flag bits (ctr[HR_CTR_FLAGS]).
#define HR_DEVF_CLOCK 1u
#define HR_DEVF_RANGE 4u
#define HR_DEVF_STALL 8u    // a batched item gave up waiting for its phase
#define HR_DEVF_LIMIT 16u   // a call site reached its record limit
#define HR_DEVF_FOLD 32u    // a block or thread id exceeded a 4-byte word's field
#define HR_DEVF_MASK 64u    // a masked wave barrier named less than its caller's group

// Counter words.
#define HR_CTR_HEAD 0     // ring append index
#define HR_CTR_FLAGS 1    // warning bits
#define HR_CTR_SITES 2    // HR_SITES per-site record counters
#define HR_CTR_LOG (HR_CTR_SITES + HR_SITES)   // access-log append index
#define HR_CTR_WORDS (HR_CTR_LOG + 1)
#define HR_COUNT_SLOTS 256   // checked-access counters, spread by block

// Record appended on a transition into the race state (matches hr_race).
struct hr_race_rec {
    uint8_t space;
    uint8_t kind;
    uint16_t site;
    uint32_t region;
    uint32_t block;
    uint32_t launch;
    uint64_t index;
    uint64_t before;
    uint64_t with;
    uint32_t tid;
    uint32_t flags;
};
static_assert(sizeof(hr_race_rec) == 48, "race record is 48 bytes");

// What hooks and barriers need besides the shadow of the accessed region:
// the report ring, counters, the launch epoch and the clock limits.
struct hr_env {
    hr_race_rec* ring;
    uint32_t* ctr;                      // HR_CTR_* words
    unsigned long long* count;          // HR_COUNT_SLOTS counters, or null
    uint32_t ring_cap;
    uint32_t launch;                    // launch epoch (9 bits)
    uint32_t launch_seq;                // launch sequence number (reports)
    uint32_t bc_max;                    // last valid block-clock value
    uint32_t wc_max;                    // last valid wave-clock value
    uint32_t group;                     // wave grouping at data-dependent hook sites:
                                        // 0 off, else lanes per grouping segment
    uint32_t site_limit;                // race records per call site; 0: no limit
    uint32_t wave_bits;                 // 6: waves synchronize; s < 6: tiles of 2^s lanes
    uint32_t word4;                     // 0: 8-byte global words; else the 4-byte
                                        // word layout (hr::c::layout)
    hr_access_rec* log;                 // access log (debug), or null; only
                                        // written while count is not null
    uint32_t log_cap;
    uint32_t nested;                    // 1: tiles of 2^wave_bits lanes nested in
                                        // waves (the hr_tn hooks of hr_nested.h)
};

// Shadow layout of a region (the address-to-shadow map): the element at row
// r, column c of a row-major array `cols` elements wide has its shadow word
// at offset
//   ((r >> th) * tiles_x + (c >> tw)) << (tw + th)      (its tile)
//   | (r & (2^th - 1)) << tw | (c & (2^tw - 1))          (its place in the tile)
// so a tile of 2^tw x 2^th elements owns consecutive shadow words.  tw = th
// = 0 is the row-major identity map (offset = element index); a 1-D region
// is one row.
struct hr_lay {
    uint32_t cols;      // elements per row
    uint32_t tiles_x;   // tiles per row of tiles: ceil(cols / 2^tw)
    uint32_t tw, th;    // log2 of the tile's width and height
};

__host__ __device__ __forceinline__ uint64_t hr_lay_off2(const hr_lay& L, uint32_t r, uint32_t c)
{
    return ((((uint64_t)(r >> L.th) * L.tiles_x + (c >> L.tw)) << (L.tw + L.th)) |
            ((uint64_t)(r & ((1u << L.th) - 1u)) << L.tw) | (uint64_t)(c & ((1u << L.tw) - 1u)));
}

// The shadow offset of element `index` (a division by cols for tiled maps).
__host__ __device__ __forceinline__ uint64_t hr_lay_off(const hr_lay& L, uint64_t index)
{
    if ((L.tw | L.th) == 0) return index;
    const uint64_t r = index / L.cols;
    return hr_lay_off2(L, (uint32_t)r, (uint32_t)(index - r * L.cols));
}

// The element index whose shadow word sits at offset `off` under map L of an
// array of `rows` rows, or UINT64_MAX for a word of a tile's padding.
__host__ __device__ __forceinline__ uint64_t hr_lay_index(const hr_lay& L, uint32_t rows,
                                                          uint64_t off)
{
    if ((L.tw | L.th) == 0) return off;
    const uint32_t tb = L.tw + L.th;
    const uint64_t tile = off >> tb, in = off & ((1ull << tb) - 1u);
    const uint64_t r = ((tile / L.tiles_x) << L.th) | (in >> L.tw);
    const uint64_t c = ((tile % L.tiles_x) << L.tw) | (in & ((1u << L.tw) - 1u));
    return (r < rows && c < L.cols) ? r * L.cols + c : UINT64_MAX;
}

// Shadow words of a region of `elems` elements (`rows` rows) under map L:
// a tiled map pads the array to whole tiles.
__host__ __device__ __forceinline__ uint64_t hr_lay_words(const hr_lay& L, uint32_t rows,
                                                          uint64_t elems)
{
    if ((L.tw | L.th) == 0) return elems;
    const uint64_t tile_rows = (rows + (1u << L.th) - 1u) >> L.th;
    return (tile_rows * L.tiles_x) << (L.tw + L.th);
}

// Plain-old-data block handed to instrumented kernels by value.
struct hr_kargs {
    hr_env env;
    uint64_t* shadow[HR_MAX_REGIONS];   // shadow words of each region (4-byte
                                        // words at this address when env.word4)
    uint64_t n_elems[HR_MAX_REGIONS];   // elements per region (0: unused)
    void* data[HR_MAX_REGIONS];         // monitored buffer of each region
    hr_lay lay[HR_MAX_REGIONS];         // address-to-shadow map of each region
};

// Per-thread checker state, kept in registers.
struct hr_thread {
    uint64_t gid;        // identity fields in global-word layout
    uint32_t lid;        // identity fields in LDS-word layout
    uint32_t block;      // logical block id
    uint32_t thread;     // thread index within the block
    uint32_t bc, wc;     // block and wave clocks
    uint32_t enabled;    // 1: checking; bit 0 clears after a clock overflow,
                         // bit 1 is set while the thread is switched off
};

__device__ __forceinline__ void hr_set_flag(const hr_env& e, uint32_t bit)
{
    __hip_atomic_fetch_or(e.ctr + HR_CTR_FLAGS, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A 4-byte word keeps block ids and thread indices modulo its field widths:
// two accessors whose ids fold together look like one, which can hide a race
// between them.  The first lane of each wave with such a thread raises the
// HR_DEVF_FOLD flag, out of line (the rare path).
__device__ __noinline__ void hr_fold_flag(uint32_t* ctr)
{
    __hip_atomic_fetch_or(ctr + HR_CTR_FLAGS, HR_DEVF_FOLD, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ hr_thread hr_thread_make(const hr_env& e, uint32_t block,
                                                    uint32_t thread)
{
    hr_thread t;
    t.block = block;
    t.thread = thread;
    t.bc = 0;
    t.wc = 0;
    t.enabled = 1;
    t.gid = hr::g::pack_id(e.launch, block, thread, 0, 0);
    t.lid = hr::l::pack_id(thread, 0, 0);
    if (e.word4) {
        const bool folded = (block & ~hr::c::block_mask(e.word4)) != 0 ||
                            (thread & ~hr::c::thread_mask(e.word4)) != 0;
        const uint64_t m = __ballot(folded);
        if (m && __lane_id() == (uint32_t)__builtin_ctzll(m)) hr_fold_flag(e.ctr);
    }
    return t;
}

// Append one access to the debug access log.
__device__ __forceinline__ void hr_log_push(hr_access_rec* log, uint32_t* ctr, uint32_t cap,
                                         uint64_t index, uint32_t region, uint32_t block,
                                         uint32_t launch_seq, uint32_t thread, uint32_t tag,
                                         uint32_t clocks, uint32_t tc = 0)
{
    const uint32_t slot =
        __hip_atomic_fetch_add(ctr + HR_CTR_LOG, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (slot >= cap) return;
    // two 16-byte stores of the 32-byte record (layout of hr_access_rec)
    uint4* p = reinterpret_cast<uint4*>(log + slot);
    p[0] = make_uint4((uint32_t)index, (uint32_t)(index >> 32), region, block);
    p[1] = make_uint4(launch_seq, (thread & 0xFFFFu) | (tag << 16), clocks, tc);
}

// Debug counting of checked accesses: one atomic per wave and hook, spread
// over HR_COUNT_SLOTS words by block to avoid a single hot address.  In the
// hooks instantiated with LOG (the kernels a context with an access log
// launches), each lane also appends its access (space, region or LDS array,
// index, kind, call site, and the thread's identity and clocks); the other
// kernels carry no logging code at all.
template <bool LOG = false>
__device__ __forceinline__ void hr_count(const hr_env& e, const hr_thread& t, uint32_t space,
                                         uint32_t region, uint64_t index, uint32_t kind,
                                         uint32_t site)
{
    if (e.count) {
        const uint64_t m = __ballot(1);
        if (__lane_id() == (uint32_t)__builtin_ctzll(m))
            __hip_atomic_fetch_add(e.count + (t.block % HR_COUNT_SLOTS),
                                   (unsigned long long)__popcll(m), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        if constexpr (LOG) {
            if (e.log)
                hr_log_push(e.log, e.ctr, e.log_cap, index, region, t.block, e.launch_seq,
                            t.thread, (space & 0xFFu) | ((kind & 0xFFu) << 8),
                            (t.bc & 0xFFu) | ((t.wc & 0xFFu) << 8) | ((site & 0xFFFFu) << 16));
        }
    }
}

// Append a race record: `before` and `with` are the two summaries whose
// accesses race (see hr_race).  The rare path: out of line, with scalar
// arguments only, so that the hooks inlined into a kernel keep neither the
// record nor the environment in registers or scratch.
__device__ __noinline__ void hr_push_rec(hr_race_rec* ring, uint32_t* ctr, uint32_t ring_cap,
                                         uint32_t site_limit, uint32_t launch_seq,
                                         uint32_t head, uint32_t region, uint32_t block,
                                         uint64_t index, uint32_t tid, uint64_t before,
                                         uint64_t with, uint32_t flags)
{
    if (site_limit) {
        const uint32_t site = head >> 16;
        const uint32_t n = __hip_atomic_fetch_add(ctr + HR_CTR_SITES + (site & (HR_SITES - 1)),
                                                  1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (n >= site_limit) {
            __hip_atomic_fetch_or(ctr + HR_CTR_FLAGS, HR_DEVF_LIMIT, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
    const uint32_t slot = __hip_atomic_fetch_add(ctr + HR_CTR_HEAD, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (slot < ring_cap) {
        // three 16-byte stores of the 48-byte record (layout of hr_race)
        uint4* p = reinterpret_cast<uint4*>(ring + slot);
        p[0] = make_uint4(head, region, block, launch_seq);
        p[1] = make_uint4((uint32_t)index, (uint32_t)(index >> 32), (uint32_t)before,
                          (uint32_t)(before >> 32));
        p[2] = make_uint4((uint32_t)with, (uint32_t)(with >> 32), tid, flags);
    }
}

__device__ __forceinline__ void hr_ring_push(const hr_env& e, uint32_t space, uint32_t region,
                                             uint32_t block, uint64_t index, uint32_t tid,
                                             uint32_t kind, uint32_t site, uint64_t before,
                                             uint64_t with, uint32_t flags)
{
    hr_push_rec(e.ring, e.ctr, e.ring_cap, e.site_limit, e.launch_seq,
                (space & 0xFFu) | ((kind & 0xFFu) << 8) | ((site & 0xFFFFu) << 16), region, block,
                index, tid, before, with, flags);
}

// Fold a summary `lost` that our exchange overwrote back into the word at
// sp, which we set to `mine`.  Each successful compare-and-swap grows the
// summary, so the loop ends after a bounded number of rounds.  Returns the
// word replaced when this fold itself created the race state (the caller
// reports it), else HR_NO_REPORT; a `lost` race state was already reported
// by whoever created it.  Out of line and with scalar arguments only: it is
// the rare path and must not make the caller spill its kernel arguments.
#define HR_NO_REPORT (~0ull)
__device__ __noinline__ uint64_t hr_fold(uint64_t* sp, uint64_t mine, uint64_t lost,
                                         uint64_t wm)
{
    uint64_t cur = mine;
    for (;;) {
        const uint64_t m = hr::g::merge(cur, lost, wm);
        if (m == cur) return HR_NO_REPORT;
        uint64_t seen = cur;
        if (__hip_atomic_compare_exchange_strong(sp, &seen, m, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return (m == hr::T_RACE && lost != hr::T_RACE) ? cur : HR_NO_REPORT;
        cur = seen;
    }
}

// Wave grouping of one hook instruction.  Lanes of a wave that run the
// same hook on the same shadow word at once (a hub vertex, a broadcast
// read) share the access kind, the block, the wave and both epochs, and
// differ only in thread; after the first two distinct threads of such a
// group a further member never changes the word.  So one owner lane applies
// itself and one other member and the rest skip their update, which turns a
// burst of same-word atomics (the contention the paper's lock-free update
// is built against, Sec. IV-B) into one.
//
// Fast path: if the words' low 32 bits rise strictly over the active lanes
// in lane order (every coalesced or strided pattern), all words differ.
// Otherwise each lane claims a hash bucket of its word in a per-wave LDS
// table; lanes whose word equals their bucket owner's word are members and
// leave a note for the owner.  Lanes whose bucket went to another word just
// update alone, so the grouping never changes the result, only the number
// of atomics.
//
// Coalescing width: lanes group only within aligned segments of `width`
// lanes (a power of two, 2..64): each segment has its own `width` buckets.
// Narrower segments do less work per hook and merge less.
#define HR_GROUP_SLOTS 1024   // one byte per thread of a block, per table
#define HR_NO_LANE 64u

__device__ __forceinline__ uint32_t hr_flat_thread()
{
    return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}

// Returns the lane of another member for an owner (HR_NO_LANE if alone) and
// sets *member for lanes whose update the owner makes.
__device__ __forceinline__ uint32_t hr_group(uint64_t word_addr, uint32_t width, bool* member)
{
    const uint32_t lane = __lane_id();
    const uint64_t act = __ballot(1);
    *member = false;
    if ((act & (act - 1)) == 0) return HR_NO_LANE;      // a single lane
    const uint64_t below = act & ((1ull << lane) - 1ull);
    const int prev = below ? 63 - __builtin_clzll(below) : (int)lane;
    const uint32_t key = (uint32_t)word_addr;
    const uint32_t pk = (uint32_t)__shfl((int)key, prev);
    if (__ballot(below != 0 && key <= pk) == 0) return HR_NO_LANE;
    __shared__ uint8_t owner_of[HR_GROUP_SLOTS];
    __shared__ uint8_t partner[HR_GROUP_SLOTS];
    const uint32_t base = hr_flat_thread() & ~63u;
    const uint32_t h = ((lane & ~(width - 1u)) |
                        ((key ^ (key >> 6) ^ (key >> 12) ^ (uint32_t)(word_addr >> 32)) &
                         (width - 1u))) & 63u;
    // Relaxed wave-scope atomics keep the compiler from forwarding a lane's
    // own store; the hardware runs a wave's LDS operations in issue order.
    __hip_atomic_store(&partner[base + lane], (uint8_t)HR_NO_LANE, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WAVEFRONT);
    __hip_atomic_store(&owner_of[base + h], (uint8_t)lane, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WAVEFRONT);             // one writer per bucket wins
    const uint32_t own =
        __hip_atomic_load(&owner_of[base + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const uint32_t olo = (uint32_t)__shfl((int)(uint32_t)word_addr, (int)own);
    const uint32_t ohi = (uint32_t)__shfl((int)(uint32_t)(word_addr >> 32), (int)own);
    const bool mem = own != lane && (((uint64_t)ohi << 32) | olo) == word_addr;
    if (mem)                                                       // one member's note wins
        __hip_atomic_store(&partner[base + own], (uint8_t)lane, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WAVEFRONT);
    const uint32_t other =
        own == lane ? (uint32_t)__hip_atomic_load(&partner[base + lane], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WAVEFRONT)
                    : HR_NO_LANE;
    *member = mem;
    return other;
}

// The record of a race completed by a global hook: the completing access
// alone or, with a group partner, the pair of lanes (if they race with each
// other) or their summary.  Out of line with scalar arguments: the rare path.
__device__ __noinline__ void hr_race8(hr_race_rec* ring, uint32_t* ctr, uint32_t ring_cap,
                                      uint32_t site_limit, uint32_t launch_seq, uint32_t head,
                                      uint32_t region, uint32_t block, uint64_t index,
                                      uint32_t thread, uint64_t gid, uint32_t k, uint64_t old,
                                      uint64_t wm, uint32_t other, uint64_t other_id)
{
    uint64_t before = old, with = hr::g::step(hr::T_INIT, gid, k, wm);
    if (other != HR_NO_LANE) {
        const uint64_t pair = hr::g::step(with, other_id, k, wm);
        if (pair == hr::T_RACE) before = hr::g::step(hr::T_INIT, other_id, k, wm);
        else with = pair;
    }
    hr_push_rec(ring, ctr, ring_cap, site_limit, launch_seq, head, region, block, index, thread,
                before, with, 0);
}

// Check one access of kind KIND (0 read, 1 write, 2 atomic) to element
// `index` (< n) of a global region whose shadow word for that element is
// shadow[off] (off: the region's address-to-shadow map applied to index);
// `region` is the id written into a race record.  GROUP marks a call site whose addresses
// depend on data (a gather or scatter); there the wave grouping runs when
// the context enables it.  Call sites with lane-affine addresses (the lanes
// of a wave touch distinct words by construction) never group.
//
// The copy-compute-publish loop of the paper's Algorithm 1, published with an
// atomic exchange instead of a compare-and-swap (on gfx950 a 64-bit exchange
// costs less than half a 64-bit compare-and-swap).  The coherent load decides
// the transition; an unchanged word costs nothing more.  If the exchange
// returns the loaded word, it acted exactly as a successful compare-and-swap.
// Otherwise it overwrote updates made since the load, and hr_fold merges
// them back.
//
// PRE: the caller loaded the word earlier (hr_check_load) and passes it as
// `pre`, to overlap that load with its other work.  Between the load and
// this call the thread passes no barrier; if another update (the thread's
// own included) landed in between, the exchange returns it and the fold
// merges it back, exactly as for an update that lands inside one hook.
// What the exchange of a check returned decides its rare paths: a race
// completed by this access is recorded; an exchange that overwrote updates
// made since the load is folded back (and a race found by the fold is
// recorded).  other / other_id: the wave-grouping partner lane, if any.
template <int KIND>
__device__ __forceinline__ void hr_settle(const hr_env& e, const hr_thread& t, uint64_t* sp,
                                          uint32_t region, uint64_t index, uint32_t site,
                                          uint64_t old, uint64_t nw, uint64_t r, uint32_t other,
                                          uint64_t other_id)
{
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    const uint64_t wm = hr::g::group_mask(e.wave_bits);
    if (nw == hr::T_RACE) {
        if (r != hr::T_RACE)
            hr_race8(e.ring, e.ctr, e.ring_cap, e.site_limit, e.launch_seq,
                     ((uint32_t)KIND << 8) | ((site & 0xFFFFu) << 16), region, t.block, index,
                     t.thread, t.gid, k, old, wm, other, other_id);
        return;
    }
    if (r != old) {
        const uint64_t before = hr_fold(sp, nw, r, wm);
        if (before != HR_NO_REPORT)
            hr_ring_push(e, 0, region, t.block, index, t.thread, KIND, site, before, r,
                         HR_RACE_FOLD);
    }
}

// The transition of a global word: the bit logic of hr::g::step, or with
// TABLE the same machine read from its flat table `tab` (hr::g::step_tab;
// a context made with HR_CFG_FSM_TABLE holds the table in device memory).
template <bool TABLE>
__device__ __forceinline__ uint64_t hr_step8(const uint16_t* tab, uint64_t old, uint64_t id,
                                             uint32_t k, uint64_t wm)
{
    if constexpr (TABLE) return hr::g::step_tab(tab, old, id, k, wm);
    else return hr::g::step(old, id, k, wm);
}

template <int KIND, bool GROUP = false, bool PRE = false, bool LOG = false, bool TABLE = false>
__device__ __forceinline__ void hr_check(const hr_env& e, const hr_thread& t, uint64_t* shadow,
                                         uint64_t n, uint32_t region, uint64_t index,
                                         uint64_t off, uint32_t site = 0, uint64_t pre = 0,
                                         const uint16_t* tab = nullptr)
{
    if (t.enabled != 1 || !shadow) return;      // thread switched off / region not monitored
    hr_count<LOG>(e, t, 0, region, index, KIND, site);
    if (index >= n) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint64_t* sp = shadow + off;
    const uint64_t wm = hr::g::group_mask(e.wave_bits);
    uint32_t other = HR_NO_LANE;
    if (GROUP && e.group && e.wave_bits == 6) {     // lanes of one tile only when tiles are waves
        bool member;
        other = hr_group((uint64_t)sp >> 3, e.group, &member);
        if (member) return;
    }
    const uint64_t old =
        PRE ? pre : __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t nw = hr_step8<TABLE>(tab, old, t.gid, k, wm);
    uint64_t other_id = 0;
    if (other != HR_NO_LANE) {
        other_id = hr::g::pack_id(e.launch, t.block, t.thread - __lane_id() + other, t.bc, t.wc);
        nw = hr_step8<TABLE>(tab, nw, other_id, k, wm);
    }
    if (nw == old) return;
    const uint64_t r = __hip_atomic_exchange(sp, nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hr_settle<KIND>(e, t, sp, region, index, site, old, nw, r, other, other_id);
}

// A check split in two at a lane-affine site: hr_check_issue publishes the
// update and returns with the exchange still in flight; hr_check_settle
// reads what it returned.  Between the two the thread may do other work
// (LDS hooks, data loads) but passes no barrier, which keeps the fold exact
// (a thread that has not settled holds back its own barriers).
struct hr_pend {
    uint64_t* sp;        // nullptr: nothing to settle
    uint64_t old, nw, r;
};

template <int KIND, bool PRE = false, bool LOG = false, bool TABLE = false>
__device__ __forceinline__ hr_pend hr_check_issue(const hr_env& e, const hr_thread& t,
                                                  uint64_t* shadow, uint64_t n, uint32_t region,
                                                  uint64_t index, uint64_t off, uint32_t site,
                                                  uint64_t pre = 0, const uint16_t* tab = nullptr)
{
    hr_pend p{nullptr, 0, 0, 0};
    if (t.enabled != 1 || !shadow) return p;
    hr_count<LOG>(e, t, 0, region, index, KIND, site);
    if (index >= n) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return p;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint64_t* sp = shadow + off;
    const uint64_t old =
        PRE ? pre : __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t nw = hr_step8<TABLE>(tab, old, t.gid, k, hr::g::group_mask(e.wave_bits));
    if (nw == old) return p;
    p.sp = sp;
    p.old = old;
    p.nw = nw;
    p.r = __hip_atomic_exchange(sp, nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return p;
}

template <int KIND>
__device__ __forceinline__ void hr_check_settle(const hr_env& e, const hr_thread& t,
                                                const hr_pend& p, uint32_t region, uint64_t index,
                                                uint32_t site)
{
    if (p.sp) hr_settle<KIND>(e, t, p.sp, region, index, site, p.old, p.nw, p.r, HR_NO_LANE, 0);
}

// The early load of hr_check<..., PRE = true>: the shadow word of element
// `index` (at shadow[off]), or 0 when the check will not use it.
__device__ __forceinline__ uint64_t hr_check_load(const hr_thread& t, uint64_t* shadow,
                                                  uint64_t n, uint64_t index, uint64_t off)
{
    return (t.enabled == 1 && shadow && index < n)
               ? __hip_atomic_load(shadow + off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : 0;
}

// ---------------------------------------------------------------------------
// The same hooks on 4-byte global words (a context created with
// HR_CFG_WORD4; word layout hr::c, e.word4).  The transition is the 64-bit
// one written over the 32-bit fields (hr::c::step) and the merge of the
// fold path widens both words, so a 4-byte word always holds the summary
// the 64-bit machine would hold for the same accesses (block ids and thread
// indices folded to the word's fields).  Race records carry widened
// summaries.
// ---------------------------------------------------------------------------
#define HR_NO_REPORT4 (~0u)   // not a word: state numbers stop at 20

__device__ __forceinline__ uint64_t hr_id4(const hr_env& e, const hr_thread& t)
{
    return hr::c::pack_id(t.block, t.thread, t.bc, t.wc, e.word4);
}

__device__ __noinline__ uint32_t hr_fold4(uint32_t* sp, uint32_t mine, uint32_t lost, uint64_t wm,
                                          uint32_t lay)
{
    uint32_t cur = mine;
    for (;;) {
        const uint32_t m = hr::c::merge(cur, lost, wm, lay);
        if (m == cur) return HR_NO_REPORT4;
        uint32_t seen = cur;
        if (__hip_atomic_compare_exchange_strong(sp, &seen, m, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return (m == hr::T_RACE && lost != hr::T_RACE) ? cur : HR_NO_REPORT4;
        cur = seen;
    }
}

// The record of a race completed by a 4-byte hook, in the 8-byte layout.
// Out of line with scalar arguments: the rare path.
__device__ __noinline__ void hr_race4(hr_race_rec* ring, uint32_t* ctr, uint32_t ring_cap,
                                      uint32_t site_limit, uint32_t launch_seq, uint32_t head,
                                      uint32_t region, uint32_t block, uint64_t index,
                                      uint32_t thread, uint32_t bc, uint32_t wc, uint32_t k,
                                      uint32_t old, uint32_t lay, uint64_t wm, uint32_t other,
                                      uint64_t other_id)
{
    uint64_t before = hr::c::widen(old, lay);
    uint64_t with = hr::g::step(hr::T_INIT, hr::c::pack_id(block, thread, bc, wc, lay), k, wm);
    if (other != HR_NO_LANE) {
        const uint64_t pair = hr::g::step(with, other_id, k, wm);
        if (pair == hr::T_RACE) before = hr::g::step(hr::T_INIT, other_id, k, wm);
        else with = pair;
    }
    hr_push_rec(ring, ctr, ring_cap, site_limit, launch_seq, head, region, block, index, thread,
                before, with, 0);
}

template <int KIND>
__device__ __forceinline__ void hr_settle4(const hr_env& e, const hr_thread& t, uint32_t* sp,
                                           uint32_t region, uint64_t index, uint32_t site,
                                           uint32_t old, uint32_t nw, uint32_t r, uint32_t other,
                                           uint64_t other_id)
{
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    const uint64_t wm = hr::g::group_mask(e.wave_bits);
    const uint32_t lay = e.word4;
    if (nw == hr::T_RACE) {
        if (r != hr::T_RACE)
            hr_race4(e.ring, e.ctr, e.ring_cap, e.site_limit, e.launch_seq,
                     0u | ((uint32_t)KIND << 8) | ((site & 0xFFFFu) << 16), region, t.block, index,
                     t.thread, t.bc, t.wc, k, old, lay, wm, other, other_id);
        return;
    }
    if (r != old) {
        const uint32_t before = hr_fold4(sp, nw, r, wm, lay);
        if (before != HR_NO_REPORT4)
            hr_ring_push(e, 0, region, t.block, index, t.thread, KIND, site,
                         hr::c::widen(before, lay), hr::c::widen(r, lay), HR_RACE_FOLD);
    }
}

// LAY: the word layout as a compile-time constant (0: the context's, e.word4).
template <int KIND, bool GROUP = false, bool PRE = false, uint32_t LAY = 0, bool LOG = false>
__device__ __forceinline__ void hr_check4(const hr_env& e, const hr_thread& t, uint32_t* shadow,
                                          uint64_t n, uint32_t region, uint64_t index,
                                          uint64_t off, uint32_t site = 0, uint32_t pre = 0)
{
    if (t.enabled != 1 || !shadow) return;
    hr_count<LOG>(e, t, 0, region, index, KIND, site);
    if (index >= n) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint32_t* sp = shadow + off;
    const uint32_t lay = LAY ? LAY : e.word4;
    const uint64_t wm = hr::g::group_mask(e.wave_bits);
    uint32_t other = HR_NO_LANE;
    if (GROUP && e.group && e.wave_bits == 6) {
        bool member;
        other = hr_group((uint64_t)sp >> 2, e.group, &member);
        if (member) return;
    }
    const uint32_t wm4 = hr::c::group_mask(e.wave_bits, lay);
    const uint32_t old =
        PRE ? pre : __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t id = hr::c::pack_id32(t.block, t.thread, t.bc, t.wc, lay);
    uint32_t nw = hr::c::step(old, id, k, wm4, lay);
    uint64_t other_id = 0;
    if (other != HR_NO_LANE) {
        const uint32_t ot = t.thread - __lane_id() + other;
        other_id = hr::c::pack_id(t.block, ot, t.bc, t.wc, lay);
        nw = hr::c::step(nw, hr::c::pack_id32(t.block, ot, t.bc, t.wc, lay), k, wm4, lay);
    }
    if (nw == old) return;
    const uint32_t r = __hip_atomic_exchange(sp, nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hr_settle4<KIND>(e, t, sp, region, index, site, old, nw, r, other, other_id);
}

struct hr_pend4 {
    uint32_t* sp;        // nullptr: nothing to settle
    uint32_t old, nw, r;
};

template <int KIND, bool PRE = false, uint32_t LAY = 0, bool LOG = false>
__device__ __forceinline__ hr_pend4 hr_check4_issue(const hr_env& e, const hr_thread& t,
                                                    uint32_t* shadow, uint64_t n, uint32_t region,
                                                    uint64_t index, uint64_t off, uint32_t site,
                                                    uint32_t pre = 0)
{
    hr_pend4 p{nullptr, 0, 0, 0};
    if (t.enabled != 1 || !shadow) return p;
    hr_count<LOG>(e, t, 0, region, index, KIND, site);
    if (index >= n) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return p;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint32_t* sp = shadow + off;
    const uint32_t old =
        PRE ? pre : __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t lay = LAY ? LAY : e.word4;
    const uint32_t nw = hr::c::step(old, hr::c::pack_id32(t.block, t.thread, t.bc, t.wc, lay), k,
                                    hr::c::group_mask(e.wave_bits, lay), lay);
    if (nw == old) return p;
    p.sp = sp;
    p.old = old;
    p.nw = nw;
    p.r = __hip_atomic_exchange(sp, nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return p;
}

template <int KIND>
__device__ __forceinline__ void hr_check4_settle(const hr_env& e, const hr_thread& t,
                                                 const hr_pend4& p, uint32_t region,
                                                 uint64_t index, uint32_t site)
{
    if (p.sp) hr_settle4<KIND>(e, t, p.sp, region, index, site, p.old, p.nw, p.r, HR_NO_LANE, 0);
}

__device__ __forceinline__ uint32_t hr_check4_load(const hr_thread& t, uint32_t* shadow,
                                                   uint64_t n, uint64_t index, uint64_t off)
{
    return (t.enabled == 1 && shadow && index < n)
               ? __hip_atomic_load(shadow + off, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               : 0u;
}

// The same check for a region named by its kernel-argument slot (the
// context's word size decides the hook).
template <int KIND>
__device__ __forceinline__ void hr_access(const hr_kargs& a, const hr_thread& t, uint32_t region,
                                          uint64_t index, uint32_t site = 0)
{
    if (region >= HR_MAX_REGIONS) {
        if (t.enabled == 1) hr_set_flag(a.env, HR_DEVF_RANGE);
        return;
    }
    const uint64_t off = hr_lay_off(a.lay[region], index);
    if (a.env.word4)
        hr_check4<KIND, true>(a.env, t, (uint32_t*)a.shadow[region], a.n_elems[region], region,
                              index, off, site);
    else
        hr_check<KIND, true>(a.env, t, a.shadow[region], a.n_elems[region], region, index, off,
                             site);
}

// Check one access to word `index` of a block's LDS array `array_id`, whose
// 4-byte shadow words live in LDS at `sh` (n_words of them, cleared to 0 at
// block start).  LDS atomics are cheap, so this path keeps the
// compare-and-swap loop.
template <int KIND, bool LOG = false>
__device__ __forceinline__ void hr_access_lds(const hr_env& e, const hr_thread& t, uint32_t* sh,
                                              uint32_t n_words, uint32_t array_id, uint32_t index,
                                              uint32_t site = 0)
{
    if (t.enabled != 1) return;
    hr_count<LOG>(e, t, 1, array_id, index, KIND, site);
    if (index >= n_words) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint32_t* sp = sh + index;
    uint32_t old = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const uint32_t nw = hr::l::step(old, t.lid, k, hr::l::group_mask(e.wave_bits));
        if (nw == old) return;
        uint32_t seen = old;
        if (__hip_atomic_compare_exchange_strong(sp, &seen, nw, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            if (nw == hr::T_RACE)
                hr_ring_push(e, 1, array_id, t.block, index, t.thread, KIND, site, old,
                             hr::l::step(hr::T_INIT, t.lid, k), 0);   // one access: split-free
            return;
        }
        old = seen;
    }
}

// The LDS hooks of one reduction step of a thread: a read of word a, a read
// of word b, then a write of word a, with no other access of the thread in
// between.  The read and the write of word a are applied in one update (the
// order in which nothing lands between them), and the two words' loads and
// compare-and-swaps are in flight together, so that the step costs two LDS
// round trips instead of six.  Sites: read a, read b, write a.
template <bool LOG = false>
__device__ __forceinline__ void hr_lds_rrw(const hr_env& e, const hr_thread& t, uint32_t* sh,
                                           uint32_t n_words, uint32_t array_id, uint32_t a,
                                           uint32_t b, uint32_t site_ra, uint32_t site_rb,
                                           uint32_t site_wa)
{
    if (t.enabled != 1) return;
    hr_count<LOG>(e, t, 1, array_id, a, 0, site_ra);
    hr_count<LOG>(e, t, 1, array_id, b, 0, site_rb);
    hr_count<LOG>(e, t, 1, array_id, a, 1, site_wa);
    if (a >= n_words || b >= n_words) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    const uint32_t wm = hr::l::group_mask(e.wave_bits);
    const uint32_t rid = hr::l::step(hr::T_INIT, t.lid, hr::CL_R);
    const uint32_t wid = hr::l::step(hr::T_INIT, t.lid, hr::CL_X);
    uint32_t* pa = sh + a;
    uint32_t* pb = sh + b;
    uint32_t oa = __hip_atomic_load(pa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    uint32_t ob = __hip_atomic_load(pb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    bool da = false, db = false;
    while (!(da && db)) {
        const uint32_t ma = hr::l::step(oa, t.lid, hr::CL_R, wm);     // word a after the read
        const uint32_t na = hr::l::step(ma, t.lid, hr::CL_X, wm);     // and after the write
        const uint32_t nb = hr::l::step(ob, t.lid, hr::CL_R, wm);
        if (!da && na == oa) da = true;
        if (!db && nb == ob) db = true;
        uint32_t sa = oa, sb = ob;
        const bool ga = !da && __hip_atomic_compare_exchange_strong(
                                   pa, &sa, na, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        const bool gb = !db && __hip_atomic_compare_exchange_strong(
                                   pb, &sb, nb, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        if (ga) {
            da = true;
            if (ma == hr::T_RACE)
                hr_ring_push(e, 1, array_id, t.block, a, t.thread, 0, site_ra, oa, rid, 0);
            else if (na == hr::T_RACE)
                hr_ring_push(e, 1, array_id, t.block, a, t.thread, 1, site_wa, ma, wid, 0);
        } else if (!da) {
            oa = sa;
        }
        if (gb) {
            db = true;
            if (nb == hr::T_RACE)
                hr_ring_push(e, 1, array_id, t.block, b, t.thread, 0, site_rb, ob, rid, 0);
        } else if (!db) {
            ob = sb;
        }
    }
}

// Runtime-kind forms (used where the kind is data, as in the interpreter).
template <bool LOG = false, bool TABLE = false>
__device__ __forceinline__ void hr_check_k(const hr_env& e, const hr_thread& t, uint32_t kind,
                                           uint64_t* shadow, uint64_t n, uint32_t region,
                                           uint64_t index, uint64_t off, uint32_t site = 0,
                                           const uint16_t* tab = nullptr)
{
    if (e.word4) {
        uint32_t* s4 = (uint32_t*)shadow;
        if (kind == 0) hr_check4<0, true, false, 0, LOG>(e, t, s4, n, region, index, off, site);
        else if (kind == 1) hr_check4<1, true, false, 0, LOG>(e, t, s4, n, region, index, off, site);
        else hr_check4<2, true, false, 0, LOG>(e, t, s4, n, region, index, off, site);
        return;
    }
    if (kind == 0)
        hr_check<0, true, false, LOG, TABLE>(e, t, shadow, n, region, index, off, site, 0, tab);
    else if (kind == 1)
        hr_check<1, true, false, LOG, TABLE>(e, t, shadow, n, region, index, off, site, 0, tab);
    else
        hr_check<2, true, false, LOG, TABLE>(e, t, shadow, n, region, index, off, site, 0, tab);
}

template <bool LOG = false>
__device__ __forceinline__ void hr_access_lds_k(const hr_env& e, const hr_thread& t,
                                                uint32_t kind, uint32_t* sh, uint32_t n_words,
                                                uint32_t array_id, uint32_t index,
                                                uint32_t site = 0)
{
    if (kind == 0) hr_access_lds<0, LOG>(e, t, sh, n_words, array_id, index, site);
    else if (kind == 1) hr_access_lds<1, LOG>(e, t, sh, n_words, array_id, index, site);
    else hr_access_lds<2, LOG>(e, t, sh, n_words, array_id, index, site);
}

__device__ __forceinline__ void hr_retag(const hr_env& e, hr_thread& t)
{
    t.gid = hr::g::pack_id(e.launch, t.block, t.thread, t.bc, t.wc);
    t.lid = hr::l::pack_id(t.thread, t.bc, t.wc);
}

// ---------------------------------------------------------------------------
// Support for kernels rewritten by the source instrumenter
// (paper_2401_04701_amd/instrument.py): every checked subscript becomes a
// call that checks the access and returns the element's address.
// ---------------------------------------------------------------------------
struct hr_rmap {
    uint32_t id[8];   // context region of each pointer parameter of the kernel
};

// Global element base[i] of the kernel's pointer parameter `slot`; K: 0 read,
// 1 write, 2 atomic, 3 read and write (compound assignment, ++, --).
template <int K, class T>
__device__ __forceinline__ T* hr_gat(const hr_kargs& a, const hr_rmap& m, const hr_thread& t,
                                     uint32_t slot, T* base, int64_t i, uint32_t site)
{
    const uint32_t r = m.id[slot];
    if (r < HR_MAX_REGIONS) {            // else the parameter is not monitored
        if (K == 3) {
            hr_access<0>(a, t, r, (uint64_t)i, site);
            hr_access<1>(a, t, r, (uint64_t)i, site);
        } else {
            hr_access<K>(a, t, r, (uint64_t)i, site);
        }
    }
    return base + i;
}

// LDS element base[i] of the kernel's shared array `id` (n words, shadow sh).
template <int K, class T>
__device__ __forceinline__ T* hr_lat(const hr_env& e, const hr_thread& t, uint32_t* sh, uint32_t n,
                                     uint32_t id, T* base, int64_t i, uint32_t site)
{
    const uint32_t idx = (i < 0 || i > (int64_t)UINT32_MAX) ? UINT32_MAX : (uint32_t)i;
    if (K == 3) {
        hr_access_lds<0>(e, t, sh, n, id, idx, site);
        hr_access_lds<1>(e, t, sh, n, id, idx, site);
    } else {
        hr_access_lds<K>(e, t, sh, n, id, idx, site);
    }
    return base + i;
}

// The checker state of a thread of an instrumented kernel: the flat
// machine's hr_thread, or the nested machine's hr_tn (hr_nested.h).
template <class T>
__device__ T hr_start(const hr_env& e, uint32_t block, uint32_t thread);

template <>
__device__ __forceinline__ hr_thread hr_start<hr_thread>(const hr_env& e, uint32_t block,
                                                         uint32_t thread)
{
    return hr_thread_make(e, block, thread);
}

// Switch the checking of this thread's accesses off or on (the paper lets a
// tool enable or disable individual threads at run time, for instance to
// track only a representative thread of each group of symmetric threads,
// Sec. IV-A).  A switched-off thread's accesses are invisible to the
// checker; its barriers still advance its clocks, so it can be switched on
// again at any point.
__device__ __forceinline__ void hr_thread_enable(hr_thread& t, bool on)
{
    t.enabled = on ? (t.enabled & ~2u) : (t.enabled | 2u);
}

// Block barrier: every thread of the block must call it (as __syncthreads).
// Advances the block clock and restarts the wave clock (paper Sec. III-A,
// Scenario 2: the block-scalar clock BC advances at each block barrier).
__device__ __forceinline__ void hr_barrier_block(const hr_env& e, hr_thread& t)
{
    __syncthreads();
    t.bc += 1;
    t.wc = 0;
    if (t.bc > e.bc_max && (t.enabled & 1u)) {
        t.enabled &= ~1u;
        hr_set_flag(e, HR_DEVF_CLOCK);
    }
    hr_retag(e, t);
}

// Wave barrier: every lane of the wave must call it; when the context
// synchronizes tiles of 2^s lanes (hr_config.wave_bits = s < 6), every lane
// of the calling lane's tile, and it orders that tile only (a tiled
// partition's sync).  Lanes are not otherwise ordered by the checker,
// whatever the hardware does.
__device__ __forceinline__ void hr_barrier_wave(const hr_env& e, hr_thread& t)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    t.wc += 1;
    if (t.wc > e.wc_max && (t.enabled & 1u)) {
        t.enabled &= ~1u;
        hr_set_flag(e, HR_DEVF_CLOCK);
    }
    hr_retag(e, t);
}

// The level a masked wave barrier (__syncwarp(mask): the lanes named in
// `mask` synchronize) reaches for the calling thread, whose linear index in
// its block is `thread`: HR_MASK_WAVE when the mask names every lane of the
// caller's wave (a last wave of a block may be partial), HR_MASK_TILE when
// it names every lane of the caller's aligned tile of 2^wave_bits lanes,
// else HR_MASK_NONE (a mask that leaves out part of the caller's tile, or
// the caller itself).  Every lane named by one mask gets the same answer
// when the mask names whole tiles.  The paper's warp barriers (Sec. III-B)
// cover a whole warp; groups below it are the future work of Sec. VI.
enum { HR_MASK_NONE = 0, HR_MASK_TILE = 1, HR_MASK_WAVE = 2 };

__device__ __forceinline__ uint32_t hr_mask_level(const hr_env& e, uint32_t thread, uint64_t mask)
{
    const uint32_t nthreads = blockDim.x * blockDim.y * blockDim.z;
    const uint32_t lane = thread & 63u;
    const uint32_t lanes = min(64u, nthreads - (thread & ~63u));
    const uint64_t exists = lanes >= 64u ? ~0ull : ((1ull << lanes) - 1ull);
    if (!((mask >> lane) & 1ull)) return HR_MASK_NONE;
    if ((mask & exists) == exists) return HR_MASK_WAVE;
    const uint32_t s = e.wave_bits;
    if (s >= 6u) return HR_MASK_NONE;
    const uint32_t w = 1u << s;
    const uint64_t tile = (((1ull << w) - 1ull) << (lane & ~(w - 1u))) & exists;
    return (mask & tile) == tile ? HR_MASK_TILE : HR_MASK_NONE;
}

// The mask of the calling lane's aligned group of n lanes (n a power of two
// up to 64): a cooperative-groups tile of n lanes.
__device__ __forceinline__ uint64_t hr_lane_tile_mask(uint32_t n)
{
    if (n >= 64u) return ~0ull;
    return ((1ull << n) - 1ull) << (__lane_id() & ~(n - 1u));
}

// Masked wave barrier on the flat machine, whose synchronization groups are
// the context's tiles (whole waves when wave_bits is 6): a mask that covers
// the caller's group orders that group (a wider mask also orders lanes of
// other groups, which this machine cannot express: it checks as if they
// were not ordered, so it may report more, never less).  A narrower mask is
// not taken as ordering anything, and hr_report warns HR_W_PARTIAL_BARRIER.
__device__ __forceinline__ void hr_barrier_mask(const hr_env& e, hr_thread& t, uint64_t mask)
{
    if (hr_mask_level(e, t.thread, mask) != HR_MASK_NONE) {
        hr_barrier_wave(e, t);
        return;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (t.enabled == 1) hr_set_flag(e, HR_DEVF_MASK);
}
