// The 5-point Jacobi sweep: its body as a device function of one logical
// block, and its standalone kernel.  The sweep's device code lives here
// alone, so that its measured figures can be tied to these sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr_device.h"
#include "hr_hooks.h"

constexpr uint32_t JACOBI_TILE = 18;
constexpr uint32_t JACOBI_TILE_WORDS = JACOBI_TILE * JACOBI_TILE;

// One 16x16 tile (logical block lb of a grid nbx tiles wide) of the 5-point
// sweep u_new = 0.2 (c + n + s + w + e), staged through an 18x18 LDS tile.
// seeds: NULL or per-block (side << 8 | offset) entries (-1: none); a seeded
// block's edge thread also writes the neighbour-owned halo cell.
// ONE_HALO: the halo reads are checked in one hook section per wave (the
// standalone kernels); without it, in two (the batch and serving workers,
// which inline every workload body under one register budget: the proxy
// lanes' second identity would spill there).
// The synchronization of a tile's threads in jacobi_body: the hardware
// block's barrier, with the LDS shadow cleared in the body.
struct hr_block_sync {
    static constexpr bool CLEARS = true;   // the body clears its LDS shadow
    template <int CHECK>
    __device__ __forceinline__ void bar(const hr_env& e, hr_thread& t) { hr_bar<CHECK>(e, t); }
};

// The synchronization of the 256 threads (4 waves) of one tile when a
// hardware block runs several tiles side by side: a barrier of those waves
// alone, on an arrival counter in LDS, so that a tile's waves do not wait
// for the other tiles' slowest wave.  The kernel clears the LDS shadow and
// the counter, then passes one block barrier, before the body runs.  Every
// wave of the tile reaches each barrier (the body's barriers are not under
// divergent control), and all are resident with their block, so the wait
// ends; it is bounded all the same, and a wait that runs out is reported as
// a stall (HR_DEVF_STALL) and goes on.  For the checker it is the tile's
// block barrier: it advances the block clock as hr_barrier_block does.
struct hr_tile_sync {
    static constexpr bool CLEARS = false;
    static constexpr uint32_t SPIN_LIMIT = 1u << 22;
    uint32_t* arrive;     // the tile's counter in LDS, zero before the body
    uint32_t target;      // arrivals that end the next barrier
    template <int CHECK>
    __device__ __forceinline__ void bar(const hr_env& e, hr_thread& t)
    {
        target += 4u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (__lane_id() == 0)
            __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        for (uint32_t spin = 0;
             __hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target;
             ++spin) {
            if (spin >= SPIN_LIMIT) {
                hr_set_flag(e, HR_DEVF_STALL);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if constexpr (CHECK) {
            t.bc += 1;
            t.wc = 0;
            if (t.bc > e.bc_max && (t.enabled & 1u)) {
                t.enabled &= ~1u;
                hr_set_flag(e, HR_DEVF_CLOCK);
            }
            hr_retag(e, t);
        }
    }
};

template <int CHECK, class G = hr_gref, bool ONE_HALO = false, class SYNC = hr_block_sync>
__device__ void jacobi_body(const hr_env& e, const G& gold, const G& gnew,
                            const float* __restrict__ uo, float* __restrict__ un, uint32_t ny,
                            uint32_t nx, uint32_t nbx, const int32_t* __restrict__ seeds,
                            uint32_t lb, uint32_t t, float* tile, uint32_t* tsh, uint32_t lds_id,
                            SYNC sync = SYNC{})
{
    constexpr uint32_t TW = JACOBI_TILE_WORDS, TL = JACOBI_TILE;
    const uint32_t tx = t & 15u, ty = (t >> 4) & 15u;
    const uint32_t bx = lb % nbx, by = lb / nbx;
    const uint32_t gx = bx * 16u + tx, gy = by * 16u + ty;
    const bool inside = t < 256 && gx < nx && gy < ny;
    hr_thread th{};
    if constexpr (CHECK) {
        th = hr_thread_make(e, lb, t);
        if constexpr (SYNC::CLEARS) {
            if (t < 256)
                for (uint32_t i = t; i < TW; i += 256) tsh[i] = 0;
            __syncthreads();
        }
    }
    const size_t g = (size_t)gy * nx + gx;
    const uint32_t cl = (ty + 1) * TL + tx + 1;
    // An edge thread stages at most one row halo cell (north or south) and
    // one column halo cell (west or east).  The data loads are issued first,
    // so that they are in flight together with the first hook's shadow load.
    const bool hn = inside && ty == 0 && gy > 0, hs = inside && ty == 15 && gy + 1 < ny;
    const bool hw = inside && tx == 0 && gx > 0, he = inside && tx == 15 && gx + 1 < nx;
    const size_t gr = hn ? g - nx : g + nx, gc = hw ? g - 1 : g + 1;
    // LDS words of the row and column halo cells, computed where they are used
    const auto lrow = [&] { return hn ? tx + 1 : 17 * TL + tx + 1; };
    const auto lcol = [&] { return hw ? (ty + 1) * TL : (ty + 1) * TL + 17; };
    const uint32_t lr = ONE_HALO ? lrow() : 0u, lc = ONE_HALO ? lcol() : 0u;
    float vr = 0.0f, vk = 0.0f;
    if (inside) {
        const float vc = uo[g];
        vr = hn || hs ? uo[gr] : 0.0f;
        vk = hw || he ? uo[gc] : 0.0f;
        // Each global hook is settled after the LDS hook of the staging
        // store that follows it, so the LDS hook runs while the exchange is
        // in flight.  (The staging hook comes before its store: the store
        // needs the loaded value, and waiting for it waits for the exchange
        // too.)
        // The centre check is blind: it steps from the initial word and
        // exchanges without loading the word first, and the settle folds
        // back the word the exchange replaced.  A word of an earlier launch
        // (or, with 4-byte words, the cleared word) adds nothing to that
        // fold, and a neighbouring block's halo read of this launch merges
        // in as another block's access, so the result is the loaded check's;
        // the wave starts with one round trip instead of two.  (The 4-byte
        // merge is the 8-byte one on widened words.)
        const typename G::pend pc = hr_gi<0, CHECK, true>(e, th, gold, gold.at2(gy, gx, g),
                                                            HR_SITE_JACOBI_CENTRE, 0);
        hr_l<1, CHECK>(e, th, tsh, TW, lds_id, cl, HR_SITE_JACOBI_STAGE);
        tile[cl] = vc;
        hr_gs<0, CHECK>(e, th, gold, pc, g, HR_SITE_JACOBI_CENTRE);
    }
    if constexpr (!CHECK) {
        if (hn || hs) tile[ONE_HALO ? lr : lrow()] = vr;
        if (hw || he) tile[ONE_HALO ? lc : lcol()] = vk;
    } else if constexpr (!ONE_HALO) {
        if (hn || hs) {
            const uint32_t lr = lrow();
            const typename G::pend pr =
                hr_gi<0, CHECK>(e, th, gold, gold.at2(hn ? gy - 1 : gy + 1, gx, gr),
                                HR_SITE_JACOBI_HALO);
            hr_l<1, CHECK>(e, th, tsh, TW, lds_id, lr, HR_SITE_JACOBI_STAGE);
            tile[lr] = vr;
            hr_gs<0, CHECK>(e, th, gold, pr, gr, HR_SITE_JACOBI_HALO);
        }
        if (hw || he) {
            const uint32_t lc = lcol();
            const typename G::pend pk =
                hr_gi<0, CHECK>(e, th, gold, gold.at2(gy, hw ? gx - 1 : gx + 1, gc),
                                HR_SITE_JACOBI_HALO);
            hr_l<1, CHECK>(e, th, tsh, TW, lds_id, lc, HR_SITE_JACOBI_STAGE);
            tile[lc] = vk;
            hr_gs<0, CHECK>(e, th, gold, pk, gc, HR_SITE_JACOBI_HALO);
        }
    } else {
        // The halo reads are checked in one hook section, one check per
        // lane: a wave's divergent sections run one after another, so a
        // lane with two halo checks would add a section for the whole
        // wave.  A lane checks its row halo read, else its column halo read.
        // The column halo read of a corner lane that also has a row halo is
        // checked by a proxy lane with no halo of its own: lane (1,1) for
        // corner (0,0), (1,14) for (0,15), (14,1) for (15,0) and (14,14) for
        // (15,15).  It is the same access, checked with the corner thread's
        // identity before the same barrier; the proxy need not own a cell.
        bool on = hn || hs || hw || he;
        size_t ha = hn || hs ? gr : gc;
        uint32_t hy = hn ? gy - 1 : (hs ? gy + 1 : gy);
        uint32_t hx = hn || hs ? gx : (hw ? gx - 1 : gx + 1);
        hr_thread hth = th;
        if (t < 256 && (ty == 1 || ty == 14) && (tx == 1 || tx == 14)) {
            const uint32_t cy = ty == 1 ? 0u : 15u, cx = tx == 1 ? 0u : 15u;
            const uint32_t cgx = bx * 16u + cx, cgy = by * 16u + cy;
            const bool row = (cy == 0 && cgy > 0) || (cy == 15 && cgy + 1 < ny);
            const bool cw = cx == 0 && cgx > 0, ce = cx == 15 && cgx + 1 < nx;
            if (cgx < nx && cgy < ny && row && (cw || ce)) {
                const size_t cg = (size_t)cgy * nx + cgx;
                on = true;
                ha = cw ? cg - 1 : cg + 1;
                hy = cgy;
                hx = cw ? cgx - 1 : cgx + 1;
                hth = hr_thread_make(e, lb, cy * 16u + cx);
            }
        }
        if (on) {
            const typename G::pend ph = hr_gi<0, CHECK>(e, hth, gold, gold.at2(hy, hx, ha),
                                                                 HR_SITE_JACOBI_HALO);
            if (hn || hs) {
                hr_l<1, CHECK>(e, th, tsh, TW, lds_id, lr, HR_SITE_JACOBI_STAGE);
                tile[lr] = vr;
            }
            if (hw || he) {
                hr_l<1, CHECK>(e, th, tsh, TW, lds_id, lc, HR_SITE_JACOBI_STAGE);
                tile[lc] = vk;
            }
            hr_gs<0, CHECK>(e, hth, gold, ph, ha, HR_SITE_JACOBI_HALO);
        }
    }
    sync.template bar<CHECK>(e, th);
    if (inside) {
        // the output word's shadow load is in flight during the LDS reads
        const hr_el xo = gnew.at2(gy, gx, g);
        const typename G::word pre_out = hr_gload<CHECK>(th, gnew, xo);
        const float c = tile[cl];
        hr_l<0, CHECK>(e, th, tsh, TW, lds_id, cl, HR_SITE_JACOBI_TILE);
        float vn = c, vs = c, vw = c, ve = c;
        if (gy > 0) {
            vn = tile[cl - TL];
            hr_l<0, CHECK>(e, th, tsh, TW, lds_id, cl - TL, HR_SITE_JACOBI_TILE);
        }
        if (gy + 1 < ny) {
            vs = tile[cl + TL];
            hr_l<0, CHECK>(e, th, tsh, TW, lds_id, cl + TL, HR_SITE_JACOBI_TILE);
        }
        if (gx > 0) {
            vw = tile[cl - 1];
            hr_l<0, CHECK>(e, th, tsh, TW, lds_id, cl - 1, HR_SITE_JACOBI_TILE);
        }
        if (gx + 1 < nx) {
            ve = tile[cl + 1];
            hr_l<0, CHECK>(e, th, tsh, TW, lds_id, cl + 1, HR_SITE_JACOBI_TILE);
        }
        const float r = 0.2f * (c + vn + vs + vw + ve);
        un[g] = r;
        hr_gpre<1, CHECK, false>(e, th, gnew, xo, HR_SITE_JACOBI_OUT, pre_out);
        if (seeds) {
            const int32_t sd = seeds[lb];
            if (sd >= 0) {
                const uint32_t side = (uint32_t)sd >> 8, off = (uint32_t)sd & 255u;
                uint32_t sy = gy, sx = gx;   // the neighbour-owned target cell
                bool hit = false;
                if (side == 0 && ty == 0 && tx == off && gy > 0) hit = true, sy = gy - 1;
                else if (side == 1 && ty == 15 && tx == off && gy + 1 < ny) hit = true, sy = gy + 1;
                else if (side == 2 && tx == 0 && ty == off && gx > 0) hit = true, sx = gx - 1;
                else if (side == 3 && tx == 15 && ty == off && gx + 1 < nx) hit = true, sx = gx + 1;
                if (hit) {
                    const size_t tgt = (size_t)sy * nx + sx;
                    un[tgt] = r;
                    hr_g<1, CHECK>(e, th, gnew, gnew.at2(sy, sx, tgt), HR_SITE_JACOBI_SEED);
                }
            }
        }
    }
}

namespace {

// One 16 x 16 tile per hardware block, on row-major shadow maps (CHECK 0:
// plain, 1: checked).  8 waves per SIMD: the hook's scalar registers would
// otherwise cap the occupancy at 7.
template <int CHECK>
__global__ __launch_bounds__(256, 8) void k_jacobi(hr_kargs a, hr_gref gold, hr_gref gnew,
                                                const float* __restrict__ uo,
                                                float* __restrict__ un, uint32_t ny, uint32_t nx,
                                                const int32_t* __restrict__ seeds)
{
    __shared__ float tile[JACOBI_TILE_WORDS];
    __shared__ uint32_t tsh[CHECK ? JACOBI_TILE_WORDS : 1];
    using G = hr_gref_map<0, 0>;
    jacobi_body<CHECK, G, true>(a.env, G{gold}, G{gnew}, uo, un, ny, nx, gridDim.x, seeds,
                                blockIdx.y * gridDim.x + blockIdx.x, threadIdx.x, tile, tsh, 0);
}

// Four consecutive tiles per 1024-thread block, each quarter of the block
// running the tuned body of k_jacobi on its own tile (row-major maps,
// checked), for launches that share the device with other streams' work:
// 1024-thread blocks of other kernels find room as this kernel's blocks
// retire, where 256-thread blocks would take every freed slot back.
// TILE_SYNC: each quarter syncs its own waves (hr_tile_sync) after one
// block barrier at the start; else the body's barriers are the whole
// block's.  Quarters past the last tile run the body without a cell.  A
// template, so that only the sources that launch it compile it.
template <int CHECK = 1, bool TILE_SYNC = true>
__global__ __launch_bounds__(1024, 8) void k_jacobi_x4(hr_kargs a, hr_gref gold, hr_gref gnew,
                                                    const float* __restrict__ uo,
                                                    float* __restrict__ un, uint32_t ny,
                                                    uint32_t nx, uint32_t nbx, uint32_t tiles,
                                                    const int32_t* __restrict__ seeds)
{
    __shared__ float tile[4][JACOBI_TILE_WORDS];
    __shared__ uint32_t tsh[4][JACOBI_TILE_WORDS];
    __shared__ uint32_t arrive[4];
    using G = hr_gref_map<0, 0>;
    const uint32_t q = threadIdx.x >> 8;
    uint32_t lb = blockIdx.x * 4u + q, t = threadIdx.x & 255u;
    if (lb >= tiles) {
        lb = blockIdx.x * 4u;
        t = UINT32_MAX;
    }
    if constexpr (TILE_SYNC) {
        if constexpr (CHECK)
            for (uint32_t i = threadIdx.x; i < 4 * JACOBI_TILE_WORDS; i += 1024)
                tsh[i / JACOBI_TILE_WORDS][i % JACOBI_TILE_WORDS] = 0;
        if (threadIdx.x < 4) arrive[threadIdx.x] = 0;
        __syncthreads();
        jacobi_body<CHECK, G, true, hr_tile_sync>(a.env, G{gold}, G{gnew}, uo, un, ny, nx, nbx,
                                                  seeds, lb, t, tile[q], tsh[q], 0,
                                                  hr_tile_sync{&arrive[q], 0u});
    } else {
        jacobi_body<CHECK, G, true>(a.env, G{gold}, G{gnew}, uo, un, ny, nx, nbx, seeds, lb, t,
                                    tile[q], tsh[q], 0);
    }
}

// The checked sweep of k_jacobi with every global transition read from the
// flat table of the machine at `tab` (a context made with
// HR_CFG_FSM_TABLE; row-major maps).  LDS_TAB: each block first copies the
// table into its LDS (32 KiB, which leaves room for 4 blocks per compute
// unit) and reads it there (HR_CFG_FSM_TABLE_LDS).  A template, so that
// only the sources that launch it compile it.
template <int CHECK = 1, bool LDS_TAB = false>
__global__ __launch_bounds__(256, 8) void k_jacobi_tab(hr_kargs a, hr_gref gold, hr_gref gnew,
                                                    const float* __restrict__ uo,
                                                    float* __restrict__ un, uint32_t ny,
                                                    uint32_t nx, const int32_t* __restrict__ seeds,
                                                    const uint16_t* __restrict__ tab)
{
    __shared__ float tile[JACOBI_TILE_WORDS];
    __shared__ uint32_t tsh[CHECK ? JACOBI_TILE_WORDS : 1];
    using G = hr_map<hr_gref_tab, 0, 0>;
    const uint16_t* t = tab;
    if constexpr (LDS_TAB) {
        // the copy is complete before the body's first hook: the body's
        // first block barrier (after its LDS shadow clear) follows it
        __shared__ uint4 stab[sizeof(hr::g::step_table) / sizeof(uint4)];
        const uint4* src = reinterpret_cast<const uint4*>(tab);
        for (uint32_t i = threadIdx.x; i < sizeof(stab) / sizeof(uint4); i += 256) stab[i] = src[i];
        t = reinterpret_cast<const uint16_t*>(stab);
    }
    jacobi_body<CHECK, G, true>(a.env, G{hr_gref_tab{gold, t}}, G{hr_gref_tab{gnew, t}}, uo, un,
                                ny, nx, gridDim.x, seeds, blockIdx.y * gridDim.x + blockIdx.x,
                                threadIdx.x, tile, tsh, 0);
}

// The checked sweep on tiled shadow maps: both grids tiled by 2^TW x 2^TH
// (constant shifts), or TW < 0: each grid's own map, read at run time.
// CHECK 2: with the debug access log (any map; row-major maps run here too).
template <int TW, int TH, int CHECK = 1>
__global__ __launch_bounds__(256, 8) void k_jacobi_tiled(hr_kargs a, hr_gref gold, hr_gref gnew,
                                                         const float* __restrict__ uo,
                                                         float* __restrict__ un, uint32_t ny,
                                                         uint32_t nx,
                                                         const int32_t* __restrict__ seeds)
{
    __shared__ float tile[JACOBI_TILE_WORDS];
    __shared__ uint32_t tsh[JACOBI_TILE_WORDS];
    using G = hr_gref_map<TW, TH>;
    jacobi_body<CHECK, G, true>(a.env, G{gold}, G{gnew}, uo, un, ny, nx, gridDim.x, seeds,
                               blockIdx.y * gridDim.x + blockIdx.x, threadIdx.x, tile, tsh, 0);
}

// The checked sweep on 4-byte shadow words, with the word layout as a
// constant (LAY) or the context's (LAY = 0); CHECK 2 adds the access log.  With a constant layout it fits
// 8 waves per SIMD; the context-layout kernel needs a few more registers
// and runs 7.
template <uint32_t LAY, int CHECK = 1>
__global__ __launch_bounds__(256, LAY ? 8 : 7) void k_jacobi4(hr_kargs a, hr_gref4t<LAY> gold,
                                                 hr_gref4t<LAY> gnew,
                                                 const float* __restrict__ uo,
                                                 float* __restrict__ un, uint32_t ny, uint32_t nx,
                                                 const int32_t* __restrict__ seeds)
{
    __shared__ float tile[JACOBI_TILE_WORDS];
    __shared__ uint32_t tsh[JACOBI_TILE_WORDS];
    jacobi_body<CHECK, hr_gref4t<LAY>, true>(a.env, gold, gnew, uo, un, ny, nx, gridDim.x, seeds,
                                            blockIdx.y * gridDim.x + blockIdx.x, threadIdx.x,
                                            tile, tsh, 0);
}

}  // namespace
