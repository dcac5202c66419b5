"""Kernels instrumented by the source rewriter, on the GPU: the flagged sets
of the rewritten example kernels must equal the oracle's sets of the same
kernels written as access programs (tests/example_programs.py; the
reductions are the oracle's reduction models), and the rewritten kernels
must still compute their results."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from example_programs import (as_tile_groups, flagged_as, histogram_program,
                              insert_block_barrier, stencil3_program, without_tile_barriers)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr
    from paper_2401_04701_amd import examples
    torch.cuda.set_device(0)
    return torch, hr, examples


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("word4", [False, True])
@pytest.mark.parametrize("drop", [-1, 0, 4, 7, 8])
def test_instrumented_reduction(env, drop, word4):
    """Also with 4-byte global shadow words (block clock of 4 bits for the
    reduction's 9 barriers): the generic hook dispatches on the context."""
    torch, hr, ex = env
    x = si.reduce_input(si.master_seed(0) + drop)
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    say("instrumented reduction drop", drop, "word4", word4)
    kw = {"word4": True, "bc_bits": 4} if word4 else {}
    with hr.Context(**kw) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ex.launch("reduce_block", ctx, [r_in, r_out], (1,), (256,), inp, out, drop)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
    want = {(sp, {0: r_in, 1: r_out}[rg] if sp == 0 else rg, lb, ix)
            for sp, rg, lb, ix in oracle.flagged(oracle.model_reduce(drop))}
    assert got == want
    if drop < 0:
        assert (out.cpu().numpy() == x.astype(np.int64).sum()).all()


@pytest.mark.parametrize("seeded", [-1, 3, 8])
def test_instrumented_stencil(env, seeded):
    torch, hr, ex = env
    n = 256 * 8 + 100                     # nine blocks, the last one ragged
    u = torch.from_numpy(si.jacobi_grid(1, n, 5)[0].copy()).cuda()
    v = torch.zeros(n, dtype=torch.float32, device="cuda")
    say("instrumented stencil seeded block", seeded)
    with hr.Context() as ctx:
        r_u, r_v = ctx.shadow_alloc(u), ctx.shadow_alloc(v)
        ex.launch("stencil3", ctx, [r_u, r_v], (9,), (256,), u, v, n, seeded)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
    want = flagged_as(stencil3_program(n, 9, seeded), [r_u, r_v])
    assert got == want and bool(want) == (0 <= seeded < 8)
    if seeded < 0:
        h = u.cpu().numpy().astype(np.float64)
        left = np.concatenate([h[:1], h[:-1]])
        right = np.concatenate([h[1:], h[-1:]])
        assert np.allclose(v.cpu().numpy(), (left + h + right) / 3.0, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("plain", [0, 1])
def test_instrumented_histogram(env, plain):
    torch, hr, ex = env
    n, bins_n = 5000, 64
    keys_h = np.random.default_rng(si.master_seed(5)).integers(0, bins_n, n).astype(np.int32)
    keys_h[:3] = 63                       # bin 63 hit by at least 3 threads
    keys_h[keys_h == 17] = 18             # bin 17 never hit
    keys = torch.from_numpy(keys_h).cuda()
    bins = torch.zeros(bins_n, dtype=torch.int32, device="cuda")
    say("instrumented histogram plain", plain)
    with hr.Context() as ctx:
        r_k, r_b = ctx.shadow_alloc(keys), ctx.shadow_alloc(bins)
        ex.launch("histogram", ctx, [r_k, r_b], ((n + 255) // 256,), (256,), keys, bins, n, plain)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
    counts = np.bincount(keys_h, minlength=bins_n)
    want = flagged_as(histogram_program(keys_h, (n + 255) // 256, 256, plain), [r_k, r_b])
    assert got == want and bool(want) == bool(plain)
    if not plain:
        assert (bins.cpu().numpy() == counts).all()


@pytest.mark.parametrize("nested", [False, True])
@pytest.mark.parametrize("drop", [-1, 0, 3, 5, 6])
def test_instrumented_wave_barriers(env, drop, nested):
    """__syncwarp becomes the checker's wave barrier: per-wave tree sums in
    LDS race exactly where the dropped wave barrier leaves two steps in one
    wave epoch (the sub-wave reduction's closed form with 64-lane tiles)."""
    torch, hr, ex = env
    blocks = 3
    x = np.random.default_rng(7 + drop).integers(0, 1 << 20, blocks * 512, dtype=np.int32)
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
    say("instrumented wave reduction drop", drop, "nested", nested)
    # with tiles nested in waves, a whole-wave __syncwarp() is a wave barrier
    kw = {"nested_tiles": True, "wave_bits": 3} if nested else {}
    with hr.Context(**kw) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ex.launch("wave_reduce", ctx, [r_in, r_out], (blocks,), (256,), inp, out, drop)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
    prog = si.tile_reduce_program(64, blocks, 256, drop)
    assert got == flagged_as(prog, [r_in, r_out])
    if drop < 0:
        want = x.astype(np.int64).reshape(blocks, 4, 128).sum(axis=2)
        assert (out.cpu().numpy().reshape(blocks, 4, 64) == want[:, :, None]).all()


TILE_DROPS = [(-1, -1), (0, -1), (2, -1), (-1, 0), (1, 0)]


@pytest.mark.parametrize("tile", [4, 8, 16])
@pytest.mark.parametrize("threads", [64, 128])
def test_instrumented_masked_tile_barriers(env, tile, threads):
    """__syncwarp(mask of the caller's tile) and whole-wave __syncwarp() in
    one kernel (examples/tile_reduce.hip: tiles reduce with tile barriers,
    waves combine the tiles' sums with wave barriers), with barriers dropped:

    * tiles nested in waves: the tile masks are tile barriers and the full
      masks wave barriers, so the set is the oracle's nested set of the
      kernel's access program, and empty with every barrier (dropping the
      last tile step's barrier leaves no race with 4-lane tiles: that step
      and the next are lane 0's alone);
    * tiles as the only groups (wave_bits = log2 tile): both kinds order the
      caller's tile only -- the oracle's set with every barrier made a tile
      barrier (a superset: it reports cross-tile pairs the wave orders);
    * whole waves (wave_bits 6): tile masks are narrower than the group and
      order nothing, with HR_W_PARTIAL_BARRIER -- the oracle's set without
      the tile barriers."""
    torch, hr, ex = env
    blocks, waves = 3, threads // 64
    tb = tile.bit_length() - 1
    x = np.random.default_rng(11 + tile).integers(0, 1 << 20, blocks * threads * 2,
                                                  dtype=np.int32)
    inp = torch.from_numpy(x).cuda()
    for dt, dw in TILE_DROPS:
        if dw >= (64 // tile).bit_length() - 1:
            continue
        prog = si.nested_reduce_program(tile, waves, blocks, dt, dw)
        for mode in ("nested", "tiles", "waves"):
            say("instrumented tile reduction", tile, threads, dt, dw, mode)
            out = torch.zeros(blocks * threads, dtype=torch.int32, device="cuda")
            kw = {"nested": {"nested_tiles": True, "wave_bits": tb},
                  "tiles": {"wave_bits": tb}, "waves": {}}[mode]
            with hr.Context(**kw) as ctx:
                r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
                ex.launch("tile_reduce", ctx, [r_in, r_out], (blocks,), (threads,), inp, out,
                          tile, dt, dw)
                ctx.kernel_end()
                got, st = ctx.flagged(), ctx.status
            regs = [r_in, r_out]
            if mode == "nested":
                want = flagged_as(prog, regs, 64, tile)
                assert st == 0 and got == want
                if dt == dw == -1:
                    assert want == set()
            elif mode == "tiles":
                want = flagged_as(as_tile_groups(prog, tile), regs, tile)
                assert st == 0 and got == want
            else:
                want = flagged_as(without_tile_barriers(prog), regs, 64)
                assert st == hr.HR_W_PARTIAL_BARRIER and got == want
            if dt == dw == -1:
                sums = x.astype(np.int64).reshape(blocks, waves, 128).sum(axis=2)
                assert (out.cpu().numpy().reshape(blocks, waves, 64) == sums[:, :, None]).all()


@pytest.mark.parametrize("threads", [64, 128])
def test_instrumented_cooperative_groups(env, threads):
    """The two-level reduction written with cooperative groups
    (examples/cg_reduce.hip): tile.sync() of a thread_block_tile<8> is the
    8-lane tile barrier, wave.sync() of a thread_block_tile<64> the wave
    barrier, block.sync() the block barrier -- the same sets, under the
    three kinds of context, as the __syncwarp(mask) version."""
    torch, hr, ex = env
    blocks, waves, tile = 3, threads // 64, 8
    x = np.random.default_rng(5 + threads).integers(0, 1 << 20, blocks * threads * 2,
                                                    dtype=np.int32)
    inp = torch.from_numpy(x).cuda()
    for dt, dw in TILE_DROPS:
        prog = si.nested_reduce_program(tile, waves, blocks, dt, dw)
        prog = insert_block_barrier(prog, prog.launches[0].phases - 1)
        for mode in ("nested", "tiles", "waves"):
            say("instrumented cooperative groups", threads, dt, dw, mode)
            out = torch.zeros(blocks * threads, dtype=torch.int32, device="cuda")
            kw = {"nested": {"nested_tiles": True, "wave_bits": 3}, "tiles": {"wave_bits": 3},
                  "waves": {}}[mode]
            with hr.Context(**kw) as ctx:
                r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
                ex.launch("cg_reduce", ctx, [r_in, r_out], (blocks,), (threads,), inp, out, dt, dw)
                ctx.kernel_end()
                got, st = ctx.flagged(), ctx.status
            regs = [r_in, r_out]
            if mode == "nested":
                assert st == 0 and got == flagged_as(prog, regs, 64, tile)
                if dt == dw == -1:
                    assert got == set()
            elif mode == "tiles":
                assert st == 0 and got == flagged_as(as_tile_groups(prog, tile), regs, tile)
            else:
                assert st == hr.HR_W_PARTIAL_BARRIER
                assert got == flagged_as(without_tile_barriers(prog), regs, 64)
            if dt == dw == -1:
                sums = x.astype(np.int64).reshape(blocks, waves, 128).sum(axis=2)
                assert (out.cpu().numpy().reshape(blocks, waves, 64) == sums[:, :, None]).all()
