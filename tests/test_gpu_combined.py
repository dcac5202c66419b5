"""The checker's options together on the GPU: sub-wave tiles as the
synchronization groups, threads switching their monitoring off and on, wave
grouping of same-word lanes, a block order that is not the hardware's, and
word ranges small enough that lanes of one instruction share words.  The
flagged set must equal the oracle's (with waves of the tile width, on the log
of the monitored accesses) bit for bit, and every race record must name a
racing pair of that log."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
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


CASES = [
    # seed, tile, grouping, p_switch, blocks, threads, phases, gwords, lwords, permuted
    (61, 64, True, 0.2, 6, 256, 5, 8, 16, True),
    (62, 16, False, 0.2, 5, 128, 5, 32, 32, True),
    (63, 8, True, 0.1, 4, 256, 6, 4, 8, False),      # grouping is off with tiles below a wave
    (64, 32, False, 0.3, 3, 1024, 4, 64, 64, True),
    (65, 64, True, 0.05, 8, 64, 4, 2, 4, True),
]


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: f"seed{c[0]}_tile{c[1]}_g{int(c[2])}")
def test_options_together(env, cfg):
    torch, hr = env
    seed, tile, grouping, p_switch, blocks, threads, phases, gw, lw, permuted = cfg
    wb = tile.bit_length() - 1
    prog = si.random_program(seed, launches=2, blocks=blocks, threads=threads, phases=phases,
                             max_ops=2, global_regions=2, global_words=gw, lds_words=lw,
                             p_lds=0.3, scope_p=(0.2, 0.5, 0.3), wave_width=tile,
                             p_switch=p_switch)
    log = oracle.model_program(prog, tile)
    want = oracle.flagged(log.copy(), tile)
    say("options", cfg, "oracle flags", len(want))
    rng = np.random.default_rng(seed)
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context(wave_bits=wb, wave_grouping=grouping, ring_capacity=1 << 16) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            bm = None
            if permuted:                          # hardware block i runs logical block bm[i]
                bm = torch.from_numpy(rng.permutation(launch.blocks).astype(np.int32)).cuda()
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words, block_map=bm)
            ctx.kernel_end()
        recs, st = ctx.report()
    assert st == 0
    remap = {r: i for i, r in enumerate(regs)}
    keys = by_key(log)
    got = set()
    for rec in recs:
        k = record_key(rec, remap)
        assert k in keys, k
        why = record_problem(rec, keys[k], strict_with=not (grouping and wb == 6), wave_bits=wb)
        assert why is None, (k, why)
        got.add(k)
    assert got == want and len(recs) == len(want)
