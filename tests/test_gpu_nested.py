"""Tiles nested in waves on the GPU (contexts with HR_CFG_NESTED_TILES): the
interpreter runs programs mixing block, wave and tile barriers, and the
flagged set must equal the oracle's with 64-lane waves and tiles of the
context's width, bit for bit; so must the access log, tile clocks included."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

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


def run_nested(torch, hr, prog, tile, block_perm_seed=None, **kw):
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    tb = tile.bit_length() - 1
    with hr.Context(nested_tiles=True, wave_bits=tb, **kw) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            bmap = None
            if block_perm_seed is not None:
                perm = np.random.default_rng(block_perm_seed).permutation(launch.blocks)
                bmap = torch.from_numpy(perm.astype(np.int32)).cuda()
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words, block_map=bmap)
            ctx.kernel_end()
        got = ctx.flagged()
        log = ctx.access_log()[0] if kw.get("access_log") else None
        return got, ctx.status, log


NESTED = [
    # seed, blocks, threads, tile, phases, max_ops, gwords, lwords, p_lds
    (1, 2, 64, 4, 6, 2, 64, 32, 0.4),
    (2, 4, 128, 8, 5, 2, 256, 128, 0.4),
    (3, 3, 192, 16, 6, 1, 300, 96, 0.5),
    (4, 2, 256, 32, 5, 2, 512, 64, 0.3),
    (5, 6, 64, 2, 8, 1, 16, 8, 0.4),          # heavy contention, 32 tiles per wave
    (6, 2, 100, 4, 6, 2, 40, 20, 0.4),        # a partial second wave
]


@pytest.mark.parametrize("cfg", NESTED, ids=lambda c: f"seed{c[0]}_t{c[2]}_tile{c[3]}")
def test_nested_program_flagged_set(env, cfg):
    torch, hr = env
    seed, blocks, threads, tile, phases, max_ops, gw, lw, p_lds = cfg
    prog = si.random_program(9000 + seed, launches=2, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=p_lds, kind_p=(0.55, 0.2, 0.25),
                             scope_p=(0.2, 0.2, 0.15, 0.45), tile_width=tile)
    want = oracle.flagged_program(prog, 64, tile)
    say("nested program", cfg, "oracle flags", len(want))
    got, st, _ = run_nested(torch, hr, prog, tile)
    assert st == 0
    assert got == want
    got2, _, _ = run_nested(torch, hr, prog, tile, block_perm_seed=seed)
    assert got2 == want
    # the flat machine with whole waves knows no tile barrier: it treats the
    # program's tile barriers as absent and so flags at least as much
    flat = oracle.flagged_program(
        si.Program([si.Launch(l.blocks, l.threads,
                              np.where(l.scope == si.SCOPE_TILE, 0, l.scope).astype(np.uint8),
                              l.wave_mask, l.op_off, l.ops) for l in prog.launches],
                   prog.global_words, prog.lds_words))
    assert want <= flat


@pytest.mark.parametrize("tile", [4, 8, 16])
def test_nested_reduction_every_dropped_barrier(env, tile):
    """Tiles reduce their segments with tile barriers, then each wave reduces
    its tiles' sums with wave barriers: race-free with every barrier, and the
    oracle's set for each dropped tile or wave barrier."""
    torch, hr = env
    s1 = (2 * tile).bit_length() - 1
    s2 = (64 // tile).bit_length() - 1
    cases = [(-1, -1)] + [(d, -1) for d in range(s1)] + [(-1, d) for d in range(s2)]
    for dt, dw in cases:
        prog = si.nested_reduce_program(tile, 2, 3, dt, dw)
        want = oracle.flagged_program(prog, 64, tile)
        say("nested reduction", tile, dt, dw, len(want))
        got, st, _ = run_nested(torch, hr, prog, tile)
        assert st == 0 and got == want
        if dt == dw == -1:
            assert want == set()


@pytest.mark.parametrize("cfg", NESTED[:3] + NESTED[5:], ids=lambda c: f"seed{c[0]}")
def test_nested_access_log(env, cfg):
    """The device log of a nested program (block, wave and tile clocks) equals
    the oracle's model of it, as multisets."""
    torch, hr = env
    seed, blocks, threads, tile, phases, max_ops, gw, lw, p_lds = cfg
    prog = si.random_program(9100 + seed, launches=2, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=p_lds, scope_p=(0.2, 0.2, 0.15, 0.45),
                             tile_width=tile, p_switch=0.05)
    model = oracle.model_program(prog, 64, tile)
    fields = ("space", "region", "index", "kind", "launch", "block", "thread", "bc", "wc", "tc")
    say("nested log", cfg, model.shape[0], "records")
    _, st, log = run_nested(torch, hr, prog, tile, access_log=True)
    assert st == 0

    def rows(a):
        out = np.zeros(a.shape[0], dtype=[(f, np.uint64) for f in fields])
        for f in fields:
            out[f] = a[f]
        out.sort(order=list(fields))
        return out
    dev, ora = rows(log), rows(model)
    assert dev.shape == ora.shape and np.array_equal(dev, ora)


@pytest.mark.parametrize("cfg", NESTED, ids=lambda c: f"seed{c[0]}")
def test_nested_records_name_racing_pairs(env, cfg):
    """Race records of a nested context: `before` and `with`, decoded in the
    nested layout (hr_describe_nested), hold a pair of the oracle's log at
    the record's key that races with tiles nested in waves, and `with` is
    the completing access alone (thread, block, class in its tile epoch)."""
    from race_records import by_key, record_key, record_problem
    torch, hr = env
    seed, blocks, threads, tile, phases, max_ops, gw, lw, p_lds = cfg
    prog = si.random_program(9000 + seed, launches=2, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=p_lds, kind_p=(0.55, 0.2, 0.25),
                             scope_p=(0.2, 0.2, 0.15, 0.45), tile_width=tile)
    log = oracle.model_program(prog, 64, tile)
    want = oracle.flagged(log.copy(), 64, tile)
    tb = tile.bit_length() - 1
    say("nested records", cfg, "oracle flags", len(want))
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context(nested_tiles=True, wave_bits=tb) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
            ctx.kernel_end()
        recs, st = ctx.report()
    assert st == 0 and len(recs) == len(want)
    keys = by_key(log)
    region_map = {r: i for i, r in enumerate(regs)}
    seen = set()
    for rec in recs:
        k = record_key(rec, region_map)
        why = record_problem(rec, keys[k], wave_bits=tb, nested=True)
        assert why is None, (k, why, rec)
        seen.add(k)
    assert seen == want


def test_nested_mode_limits(env):
    torch, hr = env
    with pytest.raises(hr.HRError):
        hr.Context(nested_tiles=True, wave_bits=6)      # tiles must be narrower than a wave
    with pytest.raises(hr.HRError):
        hr.Context(nested_tiles=True, wave_bits=3, word4=True)
    with pytest.raises(hr.HRError):
        hr.Context(nested_tiles=True, wave_bits=3, wc_bits=5)
    u = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    v = torch.zeros_like(u)
    with hr.Context(nested_tiles=True, wave_bits=3) as ctx:
        r0, r1 = ctx.shadow_alloc(u), ctx.shadow_alloc(v)
        with pytest.raises(hr.HRError):                 # no tile level in the stencil
            ctx.jacobi_check(r0, r1, u, v, None)
    # 17 tile barriers in one wave epoch pass the 4-bit tile clock: checking
    # stops in those threads with a warning; earlier races stand
    W, R = si.KIND_W, si.KIND_R
    first = [[si.op_word(si.SPACE_GLOBAL, 0, W, 0)], [si.op_word(si.SPACE_GLOBAL, 0, R, 0)]]
    phases = [[first]] + [[[[], []]] for _ in range(17)] + \
             [[[[si.op_word(si.SPACE_GLOBAL, 0, W, 1)], [si.op_word(si.SPACE_GLOBAL, 0, W, 1)]]]]
    scopes = [si.SCOPE_TILE] * 18 + [si.SCOPE_NONE]
    # two lanes in one 2-lane tile: the first phase's write and read race
    prog = si.Program([si.build_launch(1, 2, scopes, [1] * 19, phases)], [2], 2)
    got, st, _ = run_nested(torch, hr, prog, 2)
    assert st & hr.HR_W_CLOCK_OVERFLOW
    assert got == {(0, 0, 0, 0)} and got <= oracle.flagged_program(prog, 64, 2)
