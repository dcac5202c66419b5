"""GPU parity of the 4-byte global shadow word (a context with
HR_CFG_WORD4): within the word's field widths every workload's flagged set
equals the oracle's, bit for bit, as with 8-byte words; beyond them (block
ids folded) it is a subset.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle import closed_forms as cf

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


def w4(**kw):
    return dict(word4=True, **kw)


# Field widths (wave clock, block clock, thread) for the access programs:
# up to 8 barriers of each scope and 1024 threads leave a 9-bit block field.
PROG_W4 = w4(wc_bits=4, bc_bits=4, thread_bits=10)


@pytest.mark.parametrize("drop", [-1, 0, 3, 8])
def test_word4_reduce(env, drop):
    torch, hr = env
    say("word4 reduce drop", drop)
    x = si.reduce_input(si.master_seed(0) + drop)
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    with hr.Context(**w4(bc_bits=4, count_checks=True)) as ctx:   # 10 block barriers
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out, drop=drop)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
        assert ctx.check_count() == 3069
    assert got == oracle.flagged(oracle.model_reduce(drop)) == cf.reduce_flagged(drop)


PROGRAMS = [
    # seed, launches, blocks, threads, phases, max_ops, gwords, lwords, p_lds
    (1, 2, 4, 128, 4, 2, 64, 64, 0.3),
    (2, 3, 16, 256, 5, 3, 512, 256, 0.4),
    (4, 2, 8, 1000, 4, 2, 2048, 512, 0.3),
    (7, 1, 200, 64, 8, 2, 8192, 64, 0.3),
    (8, 2, 6, 256, 4, 3, 2, 4, 0.2),           # heavy same-word contention
]


def run_program(torch, hr, prog, ctx_kwargs):
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context(**ctx_kwargs) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
            ctx.kernel_end()
        return ctx.flagged(), ctx.status


@pytest.mark.parametrize("cfg", PROGRAMS, ids=lambda c: f"seed{c[0]}_b{c[2]}_t{c[3]}")
def test_word4_program(env, cfg):
    torch, hr = env
    seed, launches, blocks, threads, phases, max_ops, gw, lw, p_lds = cfg
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=3,
                             global_words=gw, lds_words=lw, p_lds=p_lds)
    want = oracle.flagged_program(prog)
    say("word4 program", cfg, "oracle flags", len(want))
    got, st = run_program(torch, hr, prog, PROG_W4)
    assert st == 0 and got == want
    got, st = run_program(torch, hr, prog, dict(PROG_W4, wave_grouping=True))
    assert st == 0 and got == want


@pytest.mark.parametrize("cfg", [(31, 2, 2, 4, 64, 4, 2, 64, 32), (34, 32, 2, 6, 1024, 4, 1, 1024, 512),
                                 (35, 4, 2, 5, 128, 6, 3, 16, 8)],
                         ids=lambda c: f"seed{c[0]}_tile{c[1]}")
def test_word4_tile_programs(env, cfg):
    """Tiles of 2^s lanes as the synchronization groups, on 4-byte words."""
    torch, hr = env
    seed, tile, launches, blocks, threads, phases, max_ops, gw, lw = cfg
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, p_lds=0.4, scope_p=(0.2, 0.6, 0.2), wave_width=tile)
    want = oracle.flagged_program(prog, tile)
    say("word4 tile program", cfg, "oracle flags", len(want))
    got, st = run_program(torch, hr, prog, dict(PROG_W4, wave_bits=tile.bit_length() - 1))
    assert st == 0 and got == want


def test_word4_switched_off_threads(env):
    torch, hr = env
    prog = si.random_program(42, launches=2, blocks=6, threads=256, phases=4, max_ops=3,
                             global_regions=2, global_words=128, lds_words=64, p_switch=0.3)
    want = oracle.flagged_program(prog)
    say("word4 switch ops, oracle flags", len(want))
    got, st = run_program(torch, hr, prog, PROG_W4)
    assert st == 0 and got == want


def test_word4_ring_overflow_recovers_global_set(env):
    """A one-record ring over two launches: the launch-boundary clear keeps
    the race words, so the report's scan still finds every global race."""
    torch, hr = env
    prog = si.random_program(23, launches=2, blocks=16, threads=256, phases=3, max_ops=2,
                             global_regions=2, global_words=256, lds_words=64, p_lds=0.3)
    want = oracle.flagged_program(prog)
    say("word4 ring overflow")
    got, st = run_program(torch, hr, prog, dict(PROG_W4, ring_capacity=1))
    assert st & hr.HR_W_RING_OVERFLOW
    assert {k for k in got if k[0] == 0} == {k for k in want if k[0] == 0}
    assert got <= want


JACOBI = [(64, 64, 3, 6), (50, 37, 2, 5), (33, 80, 4, 8), (16, 16, 2, 0), (256, 192, 3, 20),
          (1, 1, 2, 0), (1, 40, 3, 2), (40, 1, 3, 2), (17, 17, 3, 2)]


def run_jacobi(torch, hr, ny, nx, launches, tab, ctx_kwargs, grid_seed=1, seeded_launches=None):
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, grid_seed)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = None if tab is None else torch.from_numpy(tab).cuda()
    with hr.Context(**ctx_kwargs) as ctx:
        regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]
        for L in range(launches):
            t = tab_d if seeded_launches is None or L < seeded_launches else None
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], t)
            ctx.kernel_end()
        got = ctx.flagged()
        st = ctx.status
        count = ctx.check_count() if ctx_kwargs.get("count_checks") else None
    return got, st, u, count


@pytest.mark.parametrize("ny,nx,launches,count", JACOBI)
def test_word4_jacobi(env, ny, nx, launches, count):
    torch, hr = env
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + nx, count=count)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("word4 jacobi", ny, nx, launches, count)
    got, st, u, n = run_jacobi(torch, hr, ny, nx, launches, tab, w4(count_checks=True))
    log = oracle.model_jacobi(ny, nx, launches, tab)
    assert st == 0 and n == log.shape[0]
    assert got == oracle.flagged(log) == cf.jacobi_flagged(ny, nx, launches, seeds)


def test_word4_jacobi_layout_kernels_agree(env):
    """The default widths run the stencil compiled with the word layout as a
    constant; other widths that still fit run the kernel reading the layout
    from the context.  Both give the closed form's set."""
    torch, hr = env
    ny, nx, launches = 256, 192, 3
    seeds = si.jacobi_seeds(ny, nx, 57, count=12)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, launches, seeds)
    assert want
    say("word4 layout kernels")
    for widths in ({}, {"wc_bits": 2, "bc_bits": 3, "thread_bits": 9}):
        got, st, _, _ = run_jacobi(torch, hr, ny, nx, launches, tab, w4(**widths))
        assert st == 0 and got == want, widths


def test_word4_jacobi_output_matches_plain(env):
    torch, hr = env
    ny, nx = 80, 48
    say("word4 jacobi output")
    _, _, u, _ = run_jacobi(torch, hr, ny, nx, 1, None, w4())
    ref = torch.zeros_like(u[1])
    hr.jacobi_plain(u[0], ref)
    torch.cuda.synchronize()
    assert torch.equal(u[1], ref)


def test_word4_jacobi_ring_overflow_over_launches(env):
    """Races only in the first 4 of 20 launches and a one-record ring: the
    race words survive the 19 launch-boundary clears that follow."""
    torch, hr = env
    ny, nx = 48, 48
    seeds = si.jacobi_seeds(ny, nx, 78, count=3)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, 4, seeds)
    assert len(want) > 1
    say("word4 jacobi ring overflow")
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 20, tab, w4(ring_capacity=1),
                               seeded_launches=4)
    assert st & hr.HR_W_RING_OVERFLOW
    assert got == want


def test_word4_folded_blocks_flag_a_subset(env):
    """A 3-bit block field on 16 blocks: blocks 8 apart share a folded id,
    which can hide races and never adds one, and the report says so.  The
    same grid within the field widths gives no warning."""
    torch, hr = env
    ny, nx = 64, 64
    seeds = si.jacobi_seeds(ny, nx, 91, count=10)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, 3, seeds)
    say("word4 folded blocks")
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 3, tab,
                               w4(wc_bits=6, bc_bits=8, thread_bits=10))
    assert st == hr.HR_W_FOLDED and got <= want
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 3, tab, w4(wc_bits=6, bc_bits=8, thread_bits=8))
    assert st == 0 and got == want                  # 5 block bits, 8 thread bits: exact
    say("word4 folded threads")                     # 1024 threads per block, 8 thread bits
    inp = torch.from_numpy(np.random.default_rng(2).integers(0, 9, 2048).astype(np.int32)).cuda()
    out = torch.zeros(1024, dtype=torch.int32, device="cuda")
    with hr.Context(**w4(bc_bits=4)) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out, drop=-1, n=2048, threads=1024)
        ctx.kernel_end()
        assert ctx.flagged() == set() and ctx.status == hr.HR_W_FOLDED


@pytest.mark.parametrize("scale,edges,p,tpb", [(10, 8 * 1024, 0.01, 256), (9, 4096, 0.05, 1000)])
def test_word4_labelprop(env, scale, edges, p, tpb):
    torch, hr = env
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2) + scale, p)
    n = rp.shape[0] - 1
    say("word4 labelprop", scale, edges, p, tpb)
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    with hr.Context(**w4(wc_bits=1, bc_bits=1, thread_bits=10, count_checks=True)) as ctx:
        r_lab = ctx.shadow_alloc(label)
        r_rp, r_col = ctx.shadow_alloc(rp_d), ctx.shadow_alloc(col_d)
        for L in range(3):
            ctx.labelprop_check(r_lab, label, rp_d, col_d, mask_d, tpb=tpb,
                                r_row_ptr=r_rp, r_col=r_col)
            ctx.kernel_end()
        got = ctx.flagged()
        cnt = ctx.check_count()
        assert ctx.status == 0
    log = oracle.model_labelprop(rp, col, mask, 3, tpb, monitor_csr=True)
    assert cnt == log.shape[0]
    assert got == oracle.flagged(log) == cf.labelprop_flagged(rp, col, mask)


def test_word4_executors_reject_the_context(env):
    torch, hr = env
    from paper_2401_04701_amd import jobs
    say("word4 executors")
    z = np.zeros((32, 32), np.float32)
    job = jobs.Job({"pattern": hr.HR_PAT_JACOBI, "phases": 2, "nx": 32, "ny": 32},
                   {"u0": z, "u1": z, "seed_tab": None})
    with hr.Context(**w4()) as ctx:
        with pytest.raises(hr.HRError) as e:
            hr.Batch(ctx, [job.inst])
        assert e.value.status == hr.HR_E_INVAL
        with pytest.raises(hr.HRError) as e:
            hr.serve(ctx, [job.inst], [0.0])
        assert e.value.status == hr.HR_E_INVAL


def test_word4_jacobi_full_size(env):
    """4096 x 4096 (65,536 blocks, the default 16-bit block field), 20
    launches, 66 seeded blocks: the closed form's set, as with 8-byte words,
    with half the shadow memory."""
    torch, hr = env
    ny = nx = 4096
    launches = 20
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1))
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("word4 jacobi full size", ny, nx, launches, len(seeds))
    got, st, _, n = run_jacobi(torch, hr, ny, nx, launches, tab, w4(count_checks=True),
                               grid_seed=si.master_seed(1))
    assert st == 0
    assert got == cf.jacobi_flagged(ny, nx, launches, seeds)
    lib = oracle._lib()
    per_launch = lib.orc_model_jacobi(ny, nx, 0, 1, tab.ctypes.data, 0, 256, 0, 256, None, 0)
    assert n == per_launch * launches
