"""The flat-table encoding of the state machine on the GPU (contexts with
HR_CFG_FSM_TABLE): the stencil's checked kernel and the access-program
interpreter read every global transition from the table, and their flagged
sets must equal the oracle's, bit for bit, as with the bit logic."""
import json
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle.goldens import jacobi_full_workload, key_digest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2401_04701_amd import hr
    torch.cuda.set_device(0)
    return torch, hr


def say(*a):
    print("[case]", *a, flush=True)


def run_jacobi(torch, hr, ny, nx, launches, tab, **kw):
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 3)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = torch.from_numpy(tab).cuda()
    with hr.Context(ring_capacity=1 << 20, **kw) as ctx:
        regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]
        for L in range(launches):
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], tab_d)
            ctx.kernel_end()
        got, st = ctx.flagged(), ctx.status
    remap = {regs[0]: 0, regs[1]: 1}
    return {(sp, remap[rg] if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in got}, st, u


@pytest.mark.parametrize("ny,nx,launches,count", [(50, 37, 3, 5), (64, 64, 2, 8), (17, 33, 4, 2),
                                                  (1, 40, 2, 1), (48, 80, 3, 0)])
def test_table_jacobi_equals_oracle(env, ny, nx, launches, count):
    torch, hr = env
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + ny, count=count)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("table jacobi", ny, nx, launches, count)
    got, st, u = run_jacobi(torch, hr, ny, nx, launches, tab, fsm_table=True)
    want = oracle.flagged(oracle.model_jacobi(ny, nx, launches, tab))
    assert st == 0 and got == want
    got_lds, st, _ = run_jacobi(torch, hr, ny, nx, launches, tab, fsm_table="lds")
    assert st == 0 and got_lds == want
    bits, _, ub = run_jacobi(torch, hr, ny, nx, launches, tab)
    assert bits == got
    if not count:     # race-free: the sweep's output is the bit-logic kernel's, exactly
        assert torch.equal(u[launches % 2], ub[launches % 2])


@pytest.mark.parametrize("mode", [True, "lds"])
def test_table_jacobi_full_size(env, mode):
    """4096 x 4096, 20 launches, 66 seeded blocks: the oracle's set of the
    whole job (tests/golden), as the bit-logic kernel gives it; the table in
    device memory, or copied into each block's LDS."""
    torch, hr = env
    g = json.load(open(os.path.join(GOLDEN, "jacobi_4096x4096_20launches.json")))
    ny, nx, launches, seeds, tab = jacobi_full_workload()
    say("table jacobi full size", mode)
    got, st, _ = run_jacobi(torch, hr, ny, nx, launches, tab, fsm_table=mode)
    assert st == 0 and (len(got), key_digest(got)) == (g["flagged"], g["sha256"])


PROGRAMS = [
    # seed, blocks, threads, phases, max_ops, gwords, lwords, p_lds, wave width
    (1, 4, 128, 5, 2, 64, 64, 0.3, 64),
    (2, 6, 256, 4, 3, 8, 16, 0.2, 64),        # heavy contention
    (3, 5, 192, 5, 2, 128, 64, 0.4, 16),      # tiles of 16 lanes
    (4, 3, 100, 6, 2, 40, 20, 0.4, 64),       # a partial wave
]


@pytest.mark.parametrize("cfg", PROGRAMS, ids=lambda c: f"seed{c[0]}_t{c[2]}_w{c[8]}")
def test_table_program_equals_oracle(env, cfg):
    torch, hr = env
    seed, blocks, threads, phases, max_ops, gw, lw, p_lds, ww = cfg
    prog = si.random_program(7000 + seed, launches=2, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=p_lds, wave_width=ww, p_switch=0.05)
    want = oracle.flagged_program(prog, ww)
    say("table program", cfg, len(want))
    wb = int(ww).bit_length() - 1
    for perm in (None, seed):
        data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
        with hr.Context(fsm_table=True, wave_bits=wb) as ctx:
            regs = [ctx.shadow_alloc(d) for d in data]
            for launch in prog.launches:
                bmap = None
                if perm is not None:
                    p = np.random.default_rng(perm).permutation(launch.blocks).astype(np.int32)
                    bmap = torch.from_numpy(p).cuda()
                ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words, block_map=bmap)
                ctx.kernel_end()
            got, st = ctx.flagged(), ctx.status
        remap = dict(zip(regs, range(len(regs))))
        got = {(sp, remap[rg] if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in got}
        assert st == 0 and got == want


def test_table_context_limits(env):
    torch, hr = env
    for kw in ({"word4": True}, {"nested_tiles": True, "wave_bits": 3}, {"access_log": True}):
        with pytest.raises(hr.HRError):
            hr.Context(fsm_table=True, **kw)
    x = torch.zeros(256, dtype=torch.int32, device="cuda")
    y = torch.zeros(256, dtype=torch.int32, device="cuda")
    u = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    v = torch.zeros_like(u)
    with hr.Context(fsm_table=True) as ctx:
        rx, ry = ctx.shadow_alloc(x), ctx.shadow_alloc(y)
        with pytest.raises(hr.HRError):                  # no table form of the reduction
            ctx.reduce_check(rx, ry, x, y)
        ru, rv = ctx.shadow_alloc(u, tile=(2, 2)), ctx.shadow_alloc(v, tile=(2, 2))
        with pytest.raises(hr.HRError):                  # the table kernel is row-major only
            ctx.jacobi_check(ru, rv, u, v, None)


def test_stencil_autotuner(env):
    """tune.autotune_stencil times one stencil job under every shadow map and
    transition encoding; every trial flags the oracle's set, and it names a
    best map and encoding among those it timed."""
    torch, hr = env
    from paper_2401_04701_amd import tune
    ny, nx, launches = 96, 80, 3
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + 7, count=4)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 2)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    best, trials, flagged = tune.autotune_stencil(hr, u, torch.from_numpy(tab).cuda(), launches,
                                                  reps=2)
    assert flagged == oracle.flagged(oracle.model_jacobi(ny, nx, launches, tab))
    assert {"map_" + tune.tile_name(t) for t in tune.TILES} <= set(trials)
    assert {"fsm_bits", "fsm_table", "fsm_table_lds"} <= set(trials)
    assert best["tile"] in tune.TILES and best["fsm"] in ("bits", "table", "table_lds")
