// Hook call sites of the workload bodies: each wrapper calls the device hook
// when CHECK is set and compiles to nothing in the plain kernels (CHECK 0).
// CHECK 1 is the checking kernel; CHECK 2 the same with the debug access
// log compiled in (hr_count<LOG>), for contexts made with an access log.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "hr_device.h"

// An element of a global region as a hook takes it: its index (checked
// against the region's length and reported) and the offset of its shadow
// word (the region's address-to-shadow map applied to the index).
struct hr_el {
    uint64_t index, off;
};

// A global region as the hooks see it: its shadow, length, report id and
// address-to-shadow map; hr_gref4 for a context with 4-byte words.  Bodies
// written over a region type G use G::word for a pre-loaded shadow word and
// G::pend for a split hook in flight, and name elements either by index
// (at) or, in a 2-D array, by row and column (at2, no division).
struct hr_gref {
    uint64_t* shadow;
    uint64_t n;
    uint32_t id;
    hr_lay lay;
    using word = uint64_t;
    using pend = hr_pend;
    static constexpr bool TABLE = false;   // transitions by the bit logic
    __device__ __forceinline__ const uint16_t* table() const { return nullptr; }
    __device__ __forceinline__ hr_el at(uint64_t index) const { return {index, hr_lay_off(lay, index)}; }
    __device__ __forceinline__ hr_el at2(uint32_t r, uint32_t c, uint64_t index) const
    {
        return {index, hr_lay_off2(lay, r, c)};
    }
};

// An 8-byte-word region whose hooks take their transitions from the flat
// table of the machine (hr::g::step_tab) at `tab`.
struct hr_gref_tab : hr_gref {
    const uint16_t* tab;
    static constexpr bool TABLE = true;
    __device__ __forceinline__ const uint16_t* table() const { return tab; }
};

// Overloads for the 8-byte-word region types (hr_gref and types built on it).
template <class G>
using hr_if8 = std::enable_if_t<std::is_base_of<hr_gref, G>::value, int>;

// LAY: the 4-byte word layout as a compile-time constant (0: the context's).
template <uint32_t LAY>
struct hr_gref4t {
    uint32_t* shadow;
    uint64_t n;
    uint32_t id;
    hr_lay lay;
    using word = uint32_t;
    using pend = hr_pend4;
    __device__ __forceinline__ hr_el at(uint64_t index) const { return {index, hr_lay_off(lay, index)}; }
    __device__ __forceinline__ hr_el at2(uint32_t r, uint32_t c, uint64_t index) const
    {
        return {index, hr_lay_off2(lay, r, c)};
    }
};
using hr_gref4 = hr_gref4t<0>;

// The row-major map of a region `cols` elements wide (or of a 1-D region).
__host__ __device__ __forceinline__ hr_lay hr_lay_rows(uint32_t cols)
{
    return hr_lay{cols, cols, 0u, 0u};
}

// Global hook at a lane-affine site (GROUP false) or a data-dependent one.
// Every global wrapper takes the element as an hr_el, or as an index (then
// the region's map gives the shadow offset).
template <int KIND, int CHECK, bool GROUP = false, class G, hr_if8<G> = 0>
__device__ __forceinline__ void hr_g(const hr_env& e, const hr_thread& t, const G& g, hr_el x,
                                     uint32_t site)
{
    if constexpr (CHECK)
        hr_check<KIND, GROUP, false, CHECK == 2, G::TABLE>(e, t, g.shadow, g.n, g.id, x.index,
                                                           x.off, site, 0, g.table());
}

// Global hook on a word loaded earlier by hr_gload.
template <int CHECK, class G, hr_if8<G> = 0>
__device__ __forceinline__ uint64_t hr_gload(const hr_thread& t, const G& g, hr_el x)
{
    if constexpr (CHECK) return hr_check_load(t, g.shadow, g.n, x.index, x.off);
    return 0;
}

template <int KIND, int CHECK, bool GROUP = true, class G, hr_if8<G> = 0>
__device__ __forceinline__ void hr_gpre(const hr_env& e, const hr_thread& t, const G& g, hr_el x,
                                        uint32_t site, uint64_t pre)
{
    if constexpr (CHECK)
        hr_check<KIND, GROUP, true, CHECK == 2, G::TABLE>(e, t, g.shadow, g.n, g.id, x.index,
                                                          x.off, site, pre, g.table());
}

// The two halves of a global hook at a lane-affine site (hr_check_issue /
// hr_check_settle; both take the call site); `pre` as for hr_gpre when PRE.
template <int KIND, int CHECK, bool PRE = false, class G, hr_if8<G> = 0>
__device__ __forceinline__ hr_pend hr_gi(const hr_env& e, const hr_thread& t, const G& g, hr_el x,
                                         uint32_t site, uint64_t pre = 0)
{
    if constexpr (CHECK)
        return hr_check_issue<KIND, PRE, CHECK == 2, G::TABLE>(e, t, g.shadow, g.n, g.id, x.index,
                                                               x.off, site, pre, g.table());
    return hr_pend{nullptr, 0, 0, 0};
}

template <int KIND, int CHECK, class G, hr_if8<G> = 0>
__device__ __forceinline__ void hr_gs(const hr_env& e, const hr_thread& t, const G& g,
                                      const hr_pend& p, uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check_settle<KIND>(e, t, p, g.id, index, site);
}

template <int KIND, int CHECK>
__device__ __forceinline__ void hr_l(const hr_env& e, const hr_thread& t, uint32_t* sh,
                                     uint32_t n, uint32_t id, uint32_t index, uint32_t site)
{
    if constexpr (CHECK) hr_access_lds<KIND, CHECK == 2>(e, t, sh, n, id, index, site);
}

template <int CHECK>
__device__ __forceinline__ void hr_bar(const hr_env& e, hr_thread& t)
{
    if constexpr (CHECK) hr_barrier_block(e, t);
    else __syncthreads();
}

// The global hooks on 4-byte words.
template <int KIND, int CHECK, bool GROUP = false, uint32_t LAY = 0>
__device__ __forceinline__ void hr_g(const hr_env& e, const hr_thread& t, const hr_gref4t<LAY>& g,
                                     hr_el x, uint32_t site)
{
    if constexpr (CHECK)
        hr_check4<KIND, GROUP, false, LAY, CHECK == 2>(e, t, g.shadow, g.n, g.id, x.index, x.off, site);
}

template <int CHECK, uint32_t LAY = 0>
__device__ __forceinline__ uint32_t hr_gload(const hr_thread& t, const hr_gref4t<LAY>& g, hr_el x)
{
    if constexpr (CHECK) return hr_check4_load(t, g.shadow, g.n, x.index, x.off);
    return 0;
}

template <int KIND, int CHECK, bool GROUP = true, uint32_t LAY = 0>
__device__ __forceinline__ void hr_gpre(const hr_env& e, const hr_thread& t,
                                        const hr_gref4t<LAY>& g, hr_el x, uint32_t site,
                                        uint32_t pre)
{
    if constexpr (CHECK)
        hr_check4<KIND, GROUP, true, LAY, CHECK == 2>(e, t, g.shadow, g.n, g.id, x.index, x.off, site, pre);
}

template <int KIND, int CHECK, bool PRE = false, uint32_t LAY = 0>
__device__ __forceinline__ hr_pend4 hr_gi(const hr_env& e, const hr_thread& t,
                                          const hr_gref4t<LAY>& g, hr_el x, uint32_t site,
                                          uint32_t pre = 0)
{
    if constexpr (CHECK)
        return hr_check4_issue<KIND, PRE, LAY, CHECK == 2>(e, t, g.shadow, g.n, g.id, x.index, x.off, site,
                                               pre);
    return hr_pend4{nullptr, 0, 0, 0};
}

template <int KIND, int CHECK, uint32_t LAY = 0>
__device__ __forceinline__ void hr_gs(const hr_env& e, const hr_thread& t, const hr_gref4t<LAY>& g,
                                      const hr_pend4& p, uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_check4_settle<KIND>(e, t, p, g.id, index, site);
}

// The wrappers taking an element index: G is the region's own type, so a
// region type with a compile-time map (hr_map) turns the index into its
// shadow offset without the run-time map's division.
template <int KIND, int CHECK, bool GROUP = false, class G>
__device__ __forceinline__ void hr_g(const hr_env& e, const hr_thread& t, const G& g,
                                     uint64_t index, uint32_t site)
{
    if constexpr (CHECK) hr_g<KIND, CHECK, GROUP>(e, t, g, g.at(index), site);
}

template <int CHECK, class G>
__device__ __forceinline__ typename G::word hr_gload(const hr_thread& t, const G& g,
                                                     uint64_t index)
{
    if constexpr (CHECK) return hr_gload<CHECK>(t, g, g.at(index));
    return 0;
}

template <int KIND, int CHECK, bool GROUP = true, class G>
__device__ __forceinline__ void hr_gpre(const hr_env& e, const hr_thread& t, const G& g,
                                        uint64_t index, uint32_t site, typename G::word pre)
{
    if constexpr (CHECK) hr_gpre<KIND, CHECK, GROUP>(e, t, g, g.at(index), site, pre);
}

template <int KIND, int CHECK, bool PRE = false, class G>
__device__ __forceinline__ typename G::pend hr_gi(const hr_env& e, const hr_thread& t, const G& g,
                                                  uint64_t index, uint32_t site,
                                                  typename G::word pre = 0)
{
    if constexpr (CHECK) return hr_gi<KIND, CHECK, PRE>(e, t, g, g.at(index), site, pre);
    return typename G::pend{nullptr, 0, 0, 0};
}

// A region type whose map is fixed at compile time: TW = TH = 0 is the
// row-major map (the shadow offset is the element index itself; 1-D
// regions), TW, TH > 0 tiles of 2^TW x 2^TH elements with constant shifts,
// and TW < 0 the region's own map at run time.  Base: hr_gref or
// hr_gref4t<LAY>.
template <class Base, int TW, int TH>
struct hr_map : Base {
    __device__ __forceinline__ hr_el at(uint64_t index) const
    {
        if constexpr (TW == 0 && TH == 0) return {index, index};
        else return Base::at(index);
    }
    __device__ __forceinline__ hr_el at2(uint32_t r, uint32_t c, uint64_t index) const
    {
        if constexpr (TW < 0) {
            return Base::at2(r, c, index);
        } else if constexpr (TW == 0 && TH == 0) {
            return {index, index};
        } else {
            const uint64_t tile = (uint64_t)(r >> TH) * this->lay.tiles_x + (c >> TW);
            return {index, (tile << (TW + TH)) | ((uint64_t)(r & ((1u << TH) - 1u)) << TW) |
                               (uint64_t)(c & ((1u << TW) - 1u))};
        }
    }
};
template <int TW, int TH>
using hr_gref_map = hr_map<hr_gref, TW, TH>;
// 1-D regions under the identity map
using hr_gref_1d = hr_map<hr_gref, 0, 0>;
template <uint32_t LAY>
using hr_gref4_1d = hr_map<hr_gref4t<LAY>, 0, 0>;
