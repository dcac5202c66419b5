"""The source instrumenter on the CPU: which subscripts it checks, with which
access kind, how it nests rewrites, and what it leaves unchecked (GPU runs
of the instrumented examples are in test_gpu_instrumented.py)."""
import os
import re

from paper_2401_04701_amd import instrument

EX = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                  "paper_2401_04701_amd", "examples")


def kinds(text, fn):
    return [(int(k), int(line)) for k, line in
            re.findall(fn + r"<(\d)>\(.*?, (\d+)\)\)", text)]


def test_reduction_example_sites_and_kinds():
    text, (rep,) = instrument.instrument(os.path.join(EX, "reduce_block.hip"))
    assert rep.pointer_params == ["in", "out"] and rep.shared_arrays == [("a", 512)]
    assert (rep.global_sites, rep.lds_sites, rep.barriers, rep.skipped) == (3, 5, 1, [])
    # a[t] = in[t]: LDS write, global read; a[t] += a[t + h]: read-write and read
    assert sorted(kinds(text, "hr_lat")) == [(0, 14), (0, 17), (1, 10), (1, 11), (3, 14)]
    assert sorted(kinds(text, "hr_gat")) == [(0, 10), (0, 11), (1, 17)]
    assert "__syncthreads()" not in text.split("LDS shadow cleared")[1]
    assert "hr_barrier_block(hr_a.env, hr_t)" in text
    assert "hr_launch_reduce_block" in text


def test_wave_barrier_example():
    text, (rep,) = instrument.instrument(os.path.join(EX, "wave_reduce.hip"))
    assert rep.pointer_params == ["in", "out"] and rep.shared_arrays == [("s", 512)]
    assert (rep.global_sites, rep.lds_sites, rep.barriers, rep.skipped) == (3, 6, 1, [])
    body = text.split("LDS shadow cleared")[1]
    assert "__syncwarp" not in body and "hr_barrier_block" not in body
    assert body.count("hr_barrier_mask(hr_a.env, hr_t, ~0ull)") == 1   # no mask: the whole wave
    # s[base + l] = s[base + l] + s[base + l + h]: two reads, then the write
    assert sorted(kinds(text, "hr_lat")) == [(0, 16), (0, 16), (0, 19), (1, 12), (1, 13), (1, 16)]


def test_masked_wave_barriers_and_thread_state():
    """__syncwarp(mask) keeps its mask for the checker's barrier (which takes
    the tile or wave level from it at run time); the kernel becomes a
    template over the thread state, and the launcher runs the nested-machine
    instance in contexts with nested tiles."""
    text, (rep,) = instrument.instrument(os.path.join(EX, "tile_reduce.hip"))
    assert (rep.global_sites, rep.lds_sites, rep.barriers, rep.skipped) == (3, 11, 4, [])
    body = text.split("LDS shadow cleared")[1]
    assert "__syncwarp" not in body
    assert body.count("hr_barrier_mask(hr_a.env, hr_t, (unsigned long long)(mine))") == 2
    assert body.count("hr_barrier_mask(hr_a.env, hr_t, ~0ull)") == 2
    assert "template <class hr_T>\n__global__ void tile_reduce(" in text
    assert "hr_T hr_t = hr_start<hr_T>(hr_a.env," in text
    launcher = text.split("hr_launch_tile_reduce")[1]
    assert "if (hr_a.env.nested)" in launcher
    assert "tile_reduce<hr_tn>" in launcher and "tile_reduce<hr_thread>" in launcher
    assert '#include "hr_nested.h"' in text


def test_mask_expression_is_rewritten_and_unsupported_kernels(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("""#include <hip/hip_runtime.h>
static __global__ void k(const unsigned long long* masks, const int* sel, int* out)
{
    __syncwarp(masks[threadIdx.x / 8]);
    __syncwarp((unsigned long long)sel[threadIdx.x]);
    out[threadIdx.x] = 1;
}
""")
    text, (rep,) = instrument.instrument(str(src))
    assert rep.barriers == 2 and rep.global_sites == 2
    # 8-byte elements are not checked: that mask's load stays as written
    assert "hr_barrier_mask(hr_a.env, hr_t, (unsigned long long)(masks[threadIdx.x / 8]))" in text
    assert any("masks" in x for x in rep.skipped)
    # a 4-byte element read inside the mask is checked like any other read
    assert ("hr_barrier_mask(hr_a.env, hr_t, (unsigned long long)((unsigned long long)"
            "(*hr_gat<0>(hr_a, hr_m, hr_t, 1, sel, (threadIdx.x), 5))))") in text
    assert "template <class hr_T>\nstatic __global__ void k(" in text
    bad = tmp_path / "t.hip"
    bad.write_text("""#include <hip/hip_runtime.h>
extern "C" __global__ void kc(int* out) { out[threadIdx.x] = 0; }
""")
    import pytest
    with pytest.raises(RuntimeError, match="C linkage"):
        instrument.instrument(str(bad))


def test_histogram_atomic_and_compound_kinds():
    text, (rep,) = instrument.instrument(os.path.join(EX, "histogram.hip"))
    assert sorted(kinds(text, "hr_gat")) == [(0, 10), (2, 12), (3, 11)]
    assert "atomicAdd(&(*hr_gat<2>(" in text


def test_nested_and_unsupported_subscripts(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("""#include <hip/hip_runtime.h>
__global__ void gather(const int* idx, const float* in, float* out, double* wide, int n)
{
    __shared__ float m[4][4];
    const int i = threadIdx.x;
    if (i < n) out[idx[i]] = in[idx[i] + 1] + (i ? in[i] : 0.0f);
    wide[i] = 1.0;
    m[i % 4][0] = 1.0f;
    float* p = &out[i];
    *p = 2.0f;
}
""")
    text, (rep,) = instrument.instrument(str(src))
    # out[idx[i]]: the inner idx[i] is rewritten inside the outer index
    assert "(*hr_gat<1>(hr_a, hr_m, hr_t, 2, out, ((*hr_gat<0>(hr_a, hr_m, hr_t, 0, idx, (i), 6))), 6))" in text
    assert "in, ((*hr_gat<0>(hr_a, hr_m, hr_t, 0, idx, (i), 6)) + 1), 6)" in text
    assert "(*hr_gat<0>(hr_a, hr_m, hr_t, 1, in, (i), 6))" in text        # through ?:
    assert rep.global_sites == 5 and rep.lds_sites == 0
    skipped = " ".join(rep.skipped)
    assert "wide" in skipped and "double" in skipped                      # 8-byte elements
    assert "shared m" in skipped                                          # 2-D array
    assert "line 9: out" in skipped                                       # address taken


def test_example_programs_match_their_closed_forms():
    """The access programs that give the instrumented examples' expected sets
    (through the oracle) reduce to what the kernels' text says: a plain
    histogram races on every bin hit by two threads and an atomic one on
    none; the stencil's seeded block races on the first cell of the next
    block, which that block's owner also writes."""
    import numpy as np
    import synth_inputs as si
    from example_programs import flagged_as, histogram_program, stencil3_program
    keys = np.random.default_rng(si.master_seed(5)).integers(0, 64, 700).astype(np.int32)
    keys[:3] = 63
    keys[keys == 17] = 18
    counts = np.bincount(keys, minlength=64)
    assert flagged_as(histogram_program(keys, 3, 256, 1), [7, 9]) == \
        {(0, 9, 0, int(b)) for b in np.nonzero(counts >= 2)[0]}
    assert flagged_as(histogram_program(keys, 3, 256, 0), [7, 9]) == set()
    n = 256 * 8 + 100
    for seeded in (-1, 0, 3, 7, 8):
        want = {(0, 5, 0, (seeded + 1) * 256)} if 0 <= seeded < 8 else set()
        assert flagged_as(stencil3_program(n, 9, seeded), [4, 5]) == want, seeded
    # a dropped staging barrier: the halo reads meet the neighbours' writes
    prog = stencil3_program(600, 3, -1)
    prog.launches[0].scope[0] = si.SCOPE_NONE
    assert {k for k in flagged_as(prog, [0, 1]) if k[0] == 1}


def test_tile_reduce_views_of_the_barriers():
    """The expected sets of examples/tile_reduce.hip under the three ways a
    context can take its barriers: tiles nested in waves (exact), tiles as
    the only groups (wave barriers order each tile alone) and whole waves
    (tile masks order nothing).  The coarser views only add keys, and the
    race-free kernel is race-free only when nested."""
    import oracle
    import synth_inputs as si
    from example_programs import as_tile_groups, without_tile_barriers
    for tile in (4, 8):
        for dt, dw in ((-1, -1), (0, -1), (-1, 0)):
            p = si.nested_reduce_program(tile, 2, 2, dt, dw)
            exact = oracle.flagged_program(p, 64, tile)
            tiles = oracle.flagged_program(as_tile_groups(p, tile), tile)
            waves = oracle.flagged_program(without_tile_barriers(p), 64)
            assert exact <= tiles and exact <= waves
            assert (exact == set()) == (dt == dw == -1)
            assert tiles != exact and waves != exact or dt == 0
            # without tile barriers every word of a segment's first half
            # that two lanes touch (all but word 0, lane 0's alone) races
            seg = {k[3] for k in waves if k[0] == si.SPACE_LDS and k[3] < 2 * 128}
            assert seg == {g * 2 * tile + j for g in range(128 // tile) for j in range(1, tile)}


def test_cooperative_groups_syncs():
    """sync() of a thread_block_tile<N> becomes the barrier of the calling
    lane's N-lane tile, of a thread_block the block barrier; a grid or
    coalesced group's sync stays as written and is reported."""
    text, (rep,) = instrument.instrument(os.path.join(EX, "cg_reduce.hip"))
    body = text.split("LDS shadow cleared")[1]
    assert body.count("hr_barrier_mask(hr_a.env, hr_t, hr_lane_tile_mask(8))") == 2
    assert body.count("hr_barrier_mask(hr_a.env, hr_t, hr_lane_tile_mask(64))") == 2
    assert body.count("hr_barrier_block(hr_a.env, hr_t)") == 1
    assert ".sync()" not in body and rep.barriers == 5 and rep.skipped == []


def test_cooperative_groups_unmodelled_syncs(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("""#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
namespace cg = cooperative_groups;
__global__ void k(int* out)
{
    cg::coalesced_group active = cg::coalesced_threads();
    active.sync();
    out[threadIdx.x] = 1;
}
""")
    text, (rep,) = instrument.instrument(str(src))
    assert "active.sync()" in text and rep.barriers == 0
    assert any("not modelled" in x for x in rep.skipped)
