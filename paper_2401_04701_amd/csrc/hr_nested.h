// Hooks of kernels whose waves contain tiles with their own barriers (a
// context made with HR_CFG_NESTED_TILES): the same lock-free update as the
// flat hooks of hr_device.h (paper Sec. IV-B, Algorithm 1), on the nested
// machine of hr_fsm.h (hr::n, hr::nl), whose summaries have a tile level
// between the wave and the thread.  Tile barriers are the synchronization
// below the warp that the paper leaves to future work (Sec. VI).  Only the
// kernels that run such jobs include this header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr_device.h"

// Per-thread checker state with the tile clock.
struct hr_tn {
    uint64_t gid;        // identity in the nested global-word layout
    uint32_t lid;        // identity in the nested LDS-word layout
    uint32_t block, thread;
    uint32_t bc, wc, tc; // block, wave and tile clocks
    uint32_t enabled;    // as hr_thread::enabled
};

__device__ __forceinline__ void hr_tn_retag(const hr_env& e, hr_tn& t)
{
    t.gid = hr::n::pack_id(e.launch, t.block, t.thread, t.bc, t.wc, t.tc);
    t.lid = hr::nl::pack_id(t.thread, t.bc, t.wc, t.tc);
}

__device__ __forceinline__ hr_tn hr_tn_make(const hr_env& e, uint32_t block, uint32_t thread)
{
    hr_tn t;
    t.block = block;
    t.thread = thread;
    t.bc = t.wc = t.tc = 0;
    t.enabled = 1;
    hr_tn_retag(e, t);
    return t;
}

__device__ __forceinline__ void hr_tn_clock(const hr_env& e, hr_tn& t, bool overflow)
{
    if (overflow && (t.enabled & 1u)) {
        t.enabled &= ~1u;
        hr_set_flag(e, HR_DEVF_CLOCK);
    }
    hr_tn_retag(e, t);
}

// Block barrier: every thread of the block calls it.  Restarts the wave and
// tile clocks.
__device__ __forceinline__ void hr_nbarrier_block(const hr_env& e, hr_tn& t)
{
    __syncthreads();
    t.bc += 1;
    t.wc = t.tc = 0;
    hr_tn_clock(e, t, t.bc > e.bc_max);
}

// Wave barrier: every lane of the wave calls it; orders the whole wave and
// restarts the tile clocks.
__device__ __forceinline__ void hr_nbarrier_wave(const hr_env& e, hr_tn& t)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    t.wc += 1;
    t.tc = 0;
    hr_tn_clock(e, t, t.wc > e.wc_max);
}

// Tile barrier: every lane of the calling lane's tile (2^wave_bits lanes)
// calls it; it orders that tile only.  A tile lies inside one wave, whose
// lanes run in step, so a wave-scope fence pair is its synchronization.
__device__ __forceinline__ void hr_nbarrier_tile(const hr_env& e, hr_tn& t)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    t.tc += 1;
    hr_tn_clock(e, t, t.tc >= hr::n::TC_LIMIT);
}

template <bool LOG>
__device__ __forceinline__ void hr_ncount(const hr_env& e, const hr_tn& t, uint32_t space,
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
                            (t.bc & 0xFFu) | ((t.wc & 0xFFu) << 8) | ((site & 0xFFFFu) << 16),
                            t.tc);
        }
    }
}

// Fold an overwritten summary back (as hr_fold, on the nested machine).
__device__ __noinline__ uint64_t hr_nfold(uint64_t* sp, uint64_t mine, uint64_t lost, uint64_t tm)
{
    uint64_t cur = mine;
    for (;;) {
        const uint64_t m = hr::n::merge(cur, lost, tm);
        if (m == cur) return HR_NO_REPORT;
        uint64_t seen = cur;
        if (__hip_atomic_compare_exchange_strong(sp, &seen, m, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return (m == hr::T_RACE && lost != hr::T_RACE) ? cur : HR_NO_REPORT;
        cur = seen;
    }
}

// Check one access of kind KIND to element `index` (shadow word shadow[off])
// of a global region: coherent load, nested transition, exchange, and the
// fold of updates the exchange overwrote.
template <int KIND, bool LOG = false>
__device__ __forceinline__ void hr_ncheck(const hr_env& e, const hr_tn& t, uint64_t* shadow,
                                          uint64_t n, uint32_t region, uint64_t index,
                                          uint64_t off, uint32_t site)
{
    if (t.enabled != 1 || !shadow) return;
    hr_ncount<LOG>(e, t, 0, region, index, KIND, site);
    if (index >= n) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    uint64_t* sp = shadow + off;
    const uint64_t tm = hr::n::tile_mask(e.wave_bits);
    const uint64_t old = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t nw = hr::n::step(old, t.gid, k, tm);
    if (nw == old) return;
    const uint64_t r = __hip_atomic_exchange(sp, nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t head = ((uint32_t)KIND << 8) | ((site & 0xFFFFu) << 16);
    if (nw == hr::T_RACE) {
        if (r != hr::T_RACE)
            hr_push_rec(e.ring, e.ctr, e.ring_cap, e.site_limit, e.launch_seq, head, region,
                        t.block, index, t.thread, old, hr::n::step(hr::T_INIT, t.gid, k, tm), 0);
        return;
    }
    if (r != old) {
        const uint64_t before = hr_nfold(sp, nw, r, tm);
        if (before != HR_NO_REPORT)
            hr_push_rec(e.ring, e.ctr, e.ring_cap, e.site_limit, e.launch_seq, head, region,
                        t.block, index, t.thread, before, r, HR_RACE_FOLD);
    }
}

// Check one access to word `index` of the block's LDS array `array_id`
// (4-byte nested shadow words at sh): compare-and-swap loop.
template <int KIND, bool LOG = false>
__device__ __forceinline__ void hr_naccess_lds(const hr_env& e, const hr_tn& t, uint32_t* sh,
                                               uint32_t n_words, uint32_t array_id,
                                               uint32_t index, uint32_t site)
{
    if (t.enabled != 1) return;
    hr_ncount<LOG>(e, t, 1, array_id, index, KIND, site);
    if (index >= n_words) {
        hr_set_flag(e, HR_DEVF_RANGE);
        return;
    }
    constexpr uint32_t k = KIND == 0 ? hr::CL_R : (KIND == 2 ? hr::CL_A : hr::CL_X);
    const uint32_t tm = hr::nl::tile_mask(e.wave_bits);
    uint32_t* sp = sh + index;
    uint32_t old = __hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    for (;;) {
        const uint32_t nw = hr::nl::step(old, t.lid, k, tm);
        if (nw == old) return;
        uint32_t seen = old;
        if (__hip_atomic_compare_exchange_strong(sp, &seen, nw, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            if (nw == hr::T_RACE)
                hr_ring_push(e, 1, array_id, t.block, index, t.thread, KIND, site, old,
                             hr::nl::step(hr::T_INIT, t.lid, k, tm), 0);
            return;
        }
        old = seen;
    }
}

// Runtime-kind forms, for the interpreter.
template <bool LOG = false>
__device__ __forceinline__ void hr_ncheck_k(const hr_env& e, const hr_tn& t, uint32_t kind,
                                            uint64_t* shadow, uint64_t n, uint32_t region,
                                            uint64_t index, uint64_t off, uint32_t site)
{
    if (kind == 0) hr_ncheck<0, LOG>(e, t, shadow, n, region, index, off, site);
    else if (kind == 1) hr_ncheck<1, LOG>(e, t, shadow, n, region, index, off, site);
    else hr_ncheck<2, LOG>(e, t, shadow, n, region, index, off, site);
}

template <bool LOG = false>
__device__ __forceinline__ void hr_naccess_lds_k(const hr_env& e, const hr_tn& t, uint32_t kind,
                                                 uint32_t* sh, uint32_t n_words,
                                                 uint32_t array_id, uint32_t index, uint32_t site)
{
    if (kind == 0) hr_naccess_lds<0, LOG>(e, t, sh, n_words, array_id, index, site);
    else if (kind == 1) hr_naccess_lds<1, LOG>(e, t, sh, n_words, array_id, index, site);
    else hr_naccess_lds<2, LOG>(e, t, sh, n_words, array_id, index, site);
}

// Switch the checking of this thread off or on (as hr_thread_enable).
__device__ __forceinline__ void hr_tn_enable(hr_tn& t, bool on)
{
    t.enabled = on ? (t.enabled & ~2u) : (t.enabled | 2u);
}

// ---------------------------------------------------------------------------
// Instrumented kernels on the nested machine: the rewriter's kernels are
// templates over the thread state, and these overloads make the hr_tn
// instance check with the nested hooks.
// ---------------------------------------------------------------------------
template <>
__device__ __forceinline__ hr_tn hr_start<hr_tn>(const hr_env& e, uint32_t block, uint32_t thread)
{
    return hr_tn_make(e, block, thread);
}

__device__ __forceinline__ void hr_thread_enable(hr_tn& t, bool on) { hr_tn_enable(t, on); }

__device__ __forceinline__ void hr_barrier_block(const hr_env& e, hr_tn& t)
{
    hr_nbarrier_block(e, t);
}

__device__ __forceinline__ void hr_barrier_wave(const hr_env& e, hr_tn& t)
{
    hr_nbarrier_wave(e, t);
}

// Masked wave barrier with tiles nested in waves: a mask that names the
// caller's whole wave is a wave barrier, one that names the caller's whole
// tile (and perhaps other tiles, whose mutual order this machine does not
// express: it may then report more, never less) a tile barrier; a narrower
// mask orders nothing, and hr_report warns HR_W_PARTIAL_BARRIER.
__device__ __forceinline__ void hr_barrier_mask(const hr_env& e, hr_tn& t, uint64_t mask)
{
    const uint32_t level = hr_mask_level(e, t.thread, mask);
    if (level == HR_MASK_WAVE) {
        hr_nbarrier_wave(e, t);
    } else if (level == HR_MASK_TILE) {
        hr_nbarrier_tile(e, t);
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (t.enabled == 1) hr_set_flag(e, HR_DEVF_MASK);
    }
}

// A global access through a kernel-argument region (as hr_access).
template <int KIND>
__device__ __forceinline__ void hr_naccess(const hr_kargs& a, const hr_tn& t, uint32_t region,
                                           uint64_t index, uint32_t site = 0)
{
    if (region >= HR_MAX_REGIONS) {
        if (t.enabled == 1) hr_set_flag(a.env, HR_DEVF_RANGE);
        return;
    }
    hr_ncheck<KIND>(a.env, t, a.shadow[region], a.n_elems[region], region, index,
                          hr_lay_off(a.lay[region], index), site);
}

template <int K, class T>
__device__ __forceinline__ T* hr_gat(const hr_kargs& a, const hr_rmap& m, const hr_tn& t,
                                     uint32_t slot, T* base, int64_t i, uint32_t site)
{
    const uint32_t r = m.id[slot];
    if (r < HR_MAX_REGIONS) {
        if (K == 3) {
            hr_naccess<0>(a, t, r, (uint64_t)i, site);
            hr_naccess<1>(a, t, r, (uint64_t)i, site);
        } else {
            hr_naccess<K>(a, t, r, (uint64_t)i, site);
        }
    }
    return base + i;
}

template <int K, class T>
__device__ __forceinline__ T* hr_lat(const hr_env& e, const hr_tn& t, uint32_t* sh, uint32_t n,
                                     uint32_t id, T* base, int64_t i, uint32_t site)
{
    const uint32_t idx = (i < 0 || i > (int64_t)UINT32_MAX) ? UINT32_MAX : (uint32_t)i;
    if (K == 3) {
        hr_naccess_lds<0>(e, t, sh, n, id, idx, site);
        hr_naccess_lds<1>(e, t, sh, n, id, idx, site);
    } else {
        hr_naccess_lds<K>(e, t, sh, n, id, idx, site);
    }
    return base + i;
}
