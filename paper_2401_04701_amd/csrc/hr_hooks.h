// Hook call sites of the workload bodies: each wrapper calls the device hook
// when CHECK is set and compiles to nothing in the plain kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr_device.h"

// A global region as the hooks see it: its shadow, length and report id;
// hr_gref4 for a context with 4-byte words.  Bodies written over a region
// type G use G::word for a pre-loaded shadow word and G::pend for a split
// hook in flight.
struct hr_gref {
    uint64_t* shadow;
    uint64_t n;
    uint32_t id;
    using word = uint64_t;
    using pend = hr_pend;
};

// LAY: the 4-byte word layout as a compile-time constant (0: the context's).
template <uint32_t LAY>
struct hr_gref4t {
    uint32_t* shadow;
    uint64_t n;
    uint32_t id;
    using word = uint32_t;
    using pend = hr_pend4;
};
using hr_gref4 = hr_gref4t<0>;

// Global hook at a lane-affine site (GROUP false) or a data-dependent one.
template <int KIND, bool CHECK, bool GROUP = false>
__device__ __forceinline__ void hr_g(const hr_env& e, const hr_thread& t, const hr_gref& g,
                                     uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check<KIND, GROUP>(e, t, g.shadow, g.n, g.id, index, site);
}

// Global hook on a word loaded earlier by hr_gload.
template <bool CHECK>
__device__ __forceinline__ uint64_t hr_gload(const hr_thread& t, const hr_gref& g, uint64_t index)
{
    if constexpr (CHECK) return hr_check_load(t, g.shadow, g.n, index);
    return 0;
}

template <int KIND, bool CHECK, bool GROUP = true>
__device__ __forceinline__ void hr_gpre(const hr_env& e, const hr_thread& t, const hr_gref& g,
                                        uint64_t index, uint32_t site, uint64_t pre)
{
    if constexpr (CHECK) hr_check<KIND, GROUP, true>(e, t, g.shadow, g.n, g.id, index, site, pre);
}

// The two halves of a global hook at a lane-affine site (hr_check_issue /
// hr_check_settle); `pre` as for hr_gpre when PRE.
template <int KIND, bool CHECK, bool PRE = false>
__device__ __forceinline__ hr_pend hr_gi(const hr_env& e, const hr_thread& t, const hr_gref& g,
                                         uint64_t index, uint64_t pre = 0)
{
    if constexpr (CHECK) return hr_check_issue<KIND, PRE>(e, t, g.shadow, g.n, index, pre);
    return hr_pend{nullptr, 0, 0, 0};
}

template <int KIND, bool CHECK>
__device__ __forceinline__ void hr_gs(const hr_env& e, const hr_thread& t, const hr_gref& g,
                                      const hr_pend& p, uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check_settle<KIND>(e, t, p, g.id, index, site);
}

template <int KIND, bool CHECK>
__device__ __forceinline__ void hr_l(const hr_env& e, const hr_thread& t, uint32_t* sh,
                                     uint32_t n, uint32_t id, uint32_t index, uint32_t site)
{
    if constexpr (CHECK) hr_access_lds<KIND>(e, t, sh, n, id, index, site);
}

template <bool CHECK>
__device__ __forceinline__ void hr_bar(const hr_env& e, hr_thread& t)
{
    if constexpr (CHECK) hr_barrier_block(e, t);
    else __syncthreads();
}

// The global hooks on 4-byte words.
template <int KIND, bool CHECK, bool GROUP = false, uint32_t LAY = 0>
__device__ __forceinline__ void hr_g(const hr_env& e, const hr_thread& t, const hr_gref4t<LAY>& g,
                                     uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check4<KIND, GROUP, false, LAY>(e, t, g.shadow, g.n, g.id, index, site);
}

template <bool CHECK, uint32_t LAY = 0>
__device__ __forceinline__ uint32_t hr_gload(const hr_thread& t, const hr_gref4t<LAY>& g,
                                             uint64_t index)
{
    if constexpr (CHECK) return hr_check4_load(t, g.shadow, g.n, index);
    return 0;
}

template <int KIND, bool CHECK, bool GROUP = true, uint32_t LAY = 0>
__device__ __forceinline__ void hr_gpre(const hr_env& e, const hr_thread& t,
                                        const hr_gref4t<LAY>& g, uint64_t index, uint32_t site,
                                        uint32_t pre)
{
    if constexpr (CHECK)
        hr_check4<KIND, GROUP, true, LAY>(e, t, g.shadow, g.n, g.id, index, site, pre);
}

template <int KIND, bool CHECK, bool PRE = false, uint32_t LAY = 0>
__device__ __forceinline__ hr_pend4 hr_gi(const hr_env& e, const hr_thread& t,
                                          const hr_gref4t<LAY>& g, uint64_t index,
                                          uint32_t pre = 0)
{
    if constexpr (CHECK) return hr_check4_issue<KIND, PRE, LAY>(e, t, g.shadow, g.n, index, pre);
    return hr_pend4{nullptr, 0, 0, 0};
}

template <int KIND, bool CHECK, uint32_t LAY = 0>
__device__ __forceinline__ void hr_gs(const hr_env& e, const hr_thread& t, const hr_gref4t<LAY>& g,
                                      const hr_pend4& p, uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check4_settle<KIND>(e, t, p, g.id, index, site);
}
