// Pieces shared by the batched executor and the serving executor: the
// device job descriptor, block-uniform loads, and the dispatch of one work
// item to its workload body.  A work item is `pack` consecutive logical
// blocks of one phase of one job, run side by side by one 1024-thread
// hardware block (pack = 1024 / the job's block size), so that jobs with
// small blocks still fill the hardware block's waves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr.h"
#include "hr_bodies.h"
#include "hr_device.h"

constexpr uint32_t HR_WORKER_THREADS = 1024;

struct hr_inst_dev {
    uint32_t pattern, blocks, threads, phases;
    uint32_t n, ny, nbx;
    int32_t drop;
    uint32_t done_off, lds_id;
    uint32_t pack, items;     // logical blocks per work item; work items per phase
    uint32_t lds_words;       // LDS words of one logical block
    hr_gref g0, g1;
    const void* p0;
    void* p1;
    const void* p2;
    const void* p3;
};

constexpr uint32_t ITEM_BLOCK_BITS = 22;
constexpr uint32_t ITEM_PHASE_BITS = 10;

// Values the whole worker block agrees on, moved into scalar registers.  The
// bodies' block barriers sit under branches on these values (pattern, sizes,
// dropped step); the compiler must see those branches as uniform, or its
// control-flow structurizer may place a barrier under a divergent mask.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x)
{
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
template <class T>
__device__ __forceinline__ T* unip(T* p)
{
    return (T*)uni64((uint64_t)p);
}

__device__ __forceinline__ hr_gref uni_gref(const hr_gref& g)
{
    return hr_gref{unip(g.shadow), uni64(g.n), uni(g.id),
                   hr_lay{uni(g.lay.cols), uni(g.lay.tiles_x), uni(g.lay.tw), uni(g.lay.th)}};
}

// Work item `item` of `phase`: thread group g (threads g*T .. g*T+T-1, T the
// job's block size) runs logical block item*pack + g with its own slice of
// the LDS; threads past the last group, and groups past the job's last
// block, only take part in the barriers.
//
// PATTERNS: bit p set compiles the body of pattern p in.  A kernel built for
// fewer patterns needs fewer registers; its caller gives it only jobs of
// those patterns.
constexpr uint32_t HR_ALL_PATTERNS = (1u << HR_PAT_REDUCE) | (1u << HR_PAT_JACOBI) |
                                     (1u << HR_PAT_LABELPROP);

template <uint32_t PATTERNS = HR_ALL_PATTERNS>
__device__ __forceinline__ void run_item(const hr_env& e, const hr_inst_dev& I, uint32_t phase,
                                         uint32_t item, uint32_t* smem)
{
    const uint32_t T = I.threads;
    const uint32_t g = threadIdx.x / T;
    uint32_t lb = item * I.pack + g, t = threadIdx.x - g * T;
    uint32_t* lds = smem + g * I.lds_words;
    if (g >= I.pack || lb >= I.blocks) {
        t = UINT32_MAX;
        lb = item * I.pack;
        lds = smem;
    }
    if constexpr ((PATTERNS >> HR_PAT_REDUCE) & 1u) {
        if (I.pattern == HR_PAT_REDUCE) {
            using G = hr_gref_1d;   // 1-D regions: the identity map
            reduce_body<1>(e, G{I.g0}, G{I.g1}, (const int32_t*)I.p0, (int32_t*)I.p1, I.n, T, lb,
                              t, I.drop, (int32_t*)lds, lds + I.n, I.lds_id);
            return;
        }
    }
    if constexpr ((PATTERNS >> HR_PAT_JACOBI) & 1u) {
        if (I.pattern == HR_PAT_JACOBI) {
            const bool odd = phase & 1u;
            const float* uo = (const float*)(odd ? I.p1 : I.p0);
            float* un = (float*)(odd ? I.p0 : I.p1);
            jacobi_body<1>(e, odd ? I.g1 : I.g0, odd ? I.g0 : I.g1, uo, un, I.ny, I.n, I.nbx,
                              (const int32_t*)I.p2, lb, t, (float*)lds, lds + JACOBI_TILE_WORDS,
                              I.lds_id);
            return;
        }
    }
    if constexpr ((PATTERNS >> HR_PAT_LABELPROP) & 1u) {
        if (I.pattern == HR_PAT_LABELPROP) {
            using G = hr_gref_1d;
            const G none{};
            labelprop_body<1, false, G>(e, G{I.g0}, none, none, (int32_t*)I.p0,
                                        (const int32_t*)I.p1, (const int32_t*)I.p2,
                                        (const uint8_t*)I.p3, I.n, T, lb, t);
        }
    }
}

// The descriptor as every thread of the worker block sees it, in scalar
// registers.
__device__ __forceinline__ hr_inst_dev load_uniform(const hr_inst_dev& G)
{
    hr_inst_dev I;
    I.pattern = uni(G.pattern);
    I.blocks = uni(G.blocks);
    I.threads = uni(G.threads);
    I.phases = uni(G.phases);
    I.n = uni(G.n);
    I.ny = uni(G.ny);
    I.nbx = uni(G.nbx);
    I.drop = (int32_t)uni((uint32_t)G.drop);
    I.done_off = uni(G.done_off);
    I.lds_id = uni(G.lds_id);
    I.pack = uni(G.pack);
    I.items = uni(G.items);
    I.lds_words = uni(G.lds_words);
    I.g0 = uni_gref(G.g0);
    I.g1 = uni_gref(G.g1);
    I.p0 = unip(G.p0);
    I.p1 = unip(G.p1);
    I.p2 = unip(G.p2);
    I.p3 = unip(G.p3);
    return I;
}

// Descriptor of a job whose shadow words are at sh0 / sh1; report ids r0/r1.
hr_inst_dev hr_make_inst_dev(const hr_instance& in, const size_t elems[2], uint64_t* sh0,
                             uint64_t* sh1, uint32_t r0, uint32_t r1, uint32_t done_off);
