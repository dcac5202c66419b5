"""Sub-wave synchronization on the GPU: with tiles of 2^s lanes as the
synchronization groups (hr_config.wave_bits = s), wave-scope barriers order
only their tile.  The flagged set must equal the oracle's with waves of the
tile width, bit for bit; the sub-wave tree reduction must match its closed
form for every dropped tile barrier, and its race records must be valid."""
import pytest

import oracle
import synth_inputs as si
from oracle import closed_forms as cf
from race_records import by_key, record_key, record_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr
    torch.cuda.set_device(0)
    return torch, hr


def say(*a):
    print("[case]", *a, flush=True)


def run(torch, hr, prog, wave_bits):
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context(wave_bits=wave_bits) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
            ctx.kernel_end()
        recs, st = ctx.report()
    return recs, st, regs


TILE_PROGRAMS = [
    # seed, tile, launches, blocks, threads, phases, max_ops, gwords, lwords
    (31, 2, 2, 4, 64, 4, 2, 64, 32),
    (32, 8, 2, 8, 256, 5, 2, 256, 128),
    (33, 16, 3, 3, 512, 4, 2, 512, 256),
    (34, 32, 2, 6, 1024, 4, 1, 1024, 512),
    (35, 4, 2, 5, 128, 6, 3, 16, 8),
]


@pytest.mark.parametrize("cfg", TILE_PROGRAMS, ids=lambda c: f"seed{c[0]}_tile{c[1]}")
def test_tile_programs_flagged_set(env, cfg):
    torch, hr = env
    seed, tile, launches, blocks, threads, phases, max_ops, gw, lw = cfg
    wb = tile.bit_length() - 1
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=0.4, scope_p=(0.2, 0.6, 0.2), wave_width=tile)
    want = oracle.flagged_program(prog, tile)
    say("tile program", cfg, "oracle flags", len(want))
    recs, st, regs = run(torch, hr, prog, wb)
    assert st == 0
    remap = {r: i for i, r in enumerate(regs)}
    got = {record_key(r, remap) for r in recs}
    assert got == want


@pytest.mark.parametrize("tile,blocks,threads", [(4, 3, 64), (16, 5, 256), (32, 2, 1024)])
def test_tile_reduction(env, tile, blocks, threads):
    torch, hr = env
    wb = tile.bit_length() - 1
    steps = (2 * tile).bit_length() - 1
    for drop in [-1] + list(range(steps)):
        prog = si.tile_reduce_program(tile, blocks, threads, drop)
        want = cf.tile_reduce_flagged(tile, blocks, threads, drop)
        say("tile reduction", tile, blocks, threads, "drop", drop)
        recs, st, regs = run(torch, hr, prog, wb)
        assert st == 0
        remap = {r: i for i, r in enumerate(regs)}
        assert {record_key(r, remap) for r in recs} == want
        if drop >= 0 and blocks * threads <= 256:
            keys = by_key(oracle.model_program(prog, tile))
            for r in recs:
                assert record_problem(r, keys[record_key(r, remap)], wave_bits=wb) is None
    # whole waves on the same program: a tile barrier is then a barrier of
    # the whole wave, which also orders the other tiles; the verdict of this
    # program does not change, since tiles touch disjoint segments
    prog = si.tile_reduce_program(tile, blocks, threads, 0)
    recs, st, regs = run(torch, hr, prog, 6)
    remap = {r: i for i, r in enumerate(regs)}
    assert {record_key(r, remap) for r in recs} == cf.tile_reduce_flagged(tile, blocks, threads, 0)
