"""Randomized parity of the access-program interpreter on the GPU: hundreds
of random barrier programs of random shapes (1 to 6 blocks of 2 to 300
threads, partial waves, 1 to 3 launches, up to 6 phases, small address
ranges so that conflicts are common, monitoring switched off and on,
permuted block orders), each run under one of the checker's modes -- whole
waves, tiles as the groups, tiles nested in waves, the flat-table
transition, wave grouping -- and compared with the oracle's set, bit for
bit.  The seeds are fixed, so every run checks the same cases."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

MODES = ("waves", "tiles", "nested", "table", "group")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr
    torch.cuda.set_device(0)
    return torch, hr


def case(seed):
    """One random case: (mode, program, expected set, context options)."""
    r = np.random.default_rng(seed)
    mode = MODES[int(r.integers(0, len(MODES)))]
    tile = int(r.choice([2, 4, 8, 16, 32]))
    kw = dict(launches=int(r.integers(1, 4)), blocks=int(r.integers(1, 7)),
              threads=int(r.choice([2, 7, 32, 64, 65, 100, 128, 192, 256, 300])),
              phases=int(r.integers(1, 7)), max_ops=int(r.integers(1, 4)), global_regions=2,
              global_words=int(r.choice([2, 8, 64, 300])),
              lds_words=int(r.choice([2, 8, 64])), p_lds=float(r.random() * 0.6),
              p_switch=0.03 if r.random() < 0.3 else 0.0)
    if mode == "nested":
        prog = si.random_program(seed, scope_p=(0.2, 0.2, 0.15, 0.45), tile_width=tile, **kw)
        return mode, prog, oracle.flagged_program(prog, 64, tile), \
            {"nested_tiles": True, "wave_bits": tile.bit_length() - 1}, r
    if mode == "tiles":
        prog = si.random_program(seed, wave_width=tile, **kw)
        return mode, prog, oracle.flagged_program(prog, tile), \
            {"wave_bits": tile.bit_length() - 1}, r
    prog = si.random_program(seed, **kw)
    opts = {"table": {"fsm_table": True}, "group": {"wave_grouping": True}, "waves": {}}[mode]
    return mode, prog, oracle.flagged_program(prog, 64), opts, r


@pytest.mark.parametrize("chunk", range(4))
def test_random_programs_equal_oracle(env, chunk):
    torch, hr = env
    counts = dict.fromkeys(MODES, 0)
    flagged = 0
    for i in range(150):
        seed = 0x24010470 + 1000 * chunk + i
        mode, prog, want, opts, r = case(seed)
        data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
        perm = r.random() < 0.5
        with hr.Context(**opts) as ctx:
            regs = [ctx.shadow_alloc(d) for d in data]
            for launch in prog.launches:
                bmap = None
                if perm:
                    p = r.permutation(launch.blocks).astype(np.int32)
                    bmap = torch.from_numpy(p).cuda()
                ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words, block_map=bmap)
                ctx.kernel_end()
            got, st = ctx.flagged(), ctx.status
        remap = dict(zip(regs, range(len(regs))))
        got = {(sp, remap[rg] if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in got}
        assert st == 0 and got == want, (seed, mode, st)
        counts[mode] += 1
        flagged += len(want)
    print("[case] chunk", chunk, counts, "flagged keys", flagged, flush=True)
    assert all(counts.values()) and flagged > 0
