"""Access-log identity: with the debug access log on, the accesses the GPU
hooks checked (space, region or LDS array, owning block, index, kind,
launch, block, thread, block clock, wave clock) must equal, as a multiset,
the access log the oracle models for the same program.  A hook on the wrong
word, with the wrong kind, thread or epochs, or a missing or doubled hook,
fails here even where it changes no flagged set."""
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


FIELDS = ("space", "region", "lds_block", "index", "kind", "launch", "block", "thread", "bc",
          "wc")


def oracle_rows(log):
    """The oracle's records as a sorted structured array of FIELDS."""
    out = np.zeros(log.shape[0], dtype=[(f, np.uint64) for f in FIELDS])
    for f in FIELDS:
        out[f] = log[f]
    out.sort(order=list(FIELDS))
    return out


def device_rows(recs, hr, region_map=None):
    """The device log in the same form; region_map renames context region
    ids to the program's."""
    out = np.zeros(recs.shape[0], dtype=[(f, np.uint64) for f in FIELDS])
    for f in ("space", "index", "kind", "launch", "block", "thread", "bc", "wc"):
        out[f] = recs[f]
    region = recs["region"].astype(np.uint64)
    if region_map:
        glob = recs["space"] == hr.HR_GLOBAL
        region = region.copy()
        for a, b in region_map.items():
            region[glob & (recs["region"] == a)] = b
    out["region"] = region
    out["lds_block"] = np.where(recs["space"] == hr.HR_LDS, recs["block"], 0)
    out.sort(order=list(FIELDS))
    return out


def same(dev, ora):
    assert dev.shape == ora.shape, (dev.shape, ora.shape)
    bad = np.nonzero(dev != ora)[0]
    assert bad.size == 0, (bad[:4], dev[bad[:4]], ora[bad[:4]])


@pytest.mark.parametrize("drop", [-1] + list(range(9)))
def test_reduce_access_log(env, drop):
    torch, hr = env
    x = si.reduce_input(si.master_seed(0))
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    say("reduce log, drop", drop)
    with hr.Context(access_log=True) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out, drop=drop)
        ctx.kernel_end()
        recs, st = ctx.access_log()
        assert st == 0
        assert ctx.check_count() == recs.shape[0]
    same(device_rows(recs, hr), oracle_rows(oracle.model_reduce(drop)))


@pytest.mark.parametrize("ny,nx,launches,count,tile,word4", [
    (50, 37, 2, 5, None, False), (33, 80, 3, 8, None, False), (17, 17, 3, 2, None, False),
    (64, 48, 2, 4, (2, 2), False), (40, 70, 2, 3, None, True), (1, 40, 2, 1, None, False)])
def test_jacobi_access_log(env, ny, nx, launches, count, tile, word4):
    torch, hr = env
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + nx, count=count)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 1)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = torch.from_numpy(tab).cuda()
    say("jacobi log", ny, nx, launches, count, tile, word4)
    with hr.Context(access_log=True, word4=word4) as ctx:
        regs = [ctx.shadow_alloc(u[0], tile=tile), ctx.shadow_alloc(u[1], tile=tile)]
        for L in range(launches):
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], tab_d)
            ctx.kernel_end()
        recs, st = ctx.access_log()
        assert st == 0
    same(device_rows(recs, hr), oracle_rows(oracle.model_jacobi(ny, nx, launches, tab)))


@pytest.mark.parametrize("grouping", [False, True])
def test_labelprop_access_log(env, grouping):
    """Scale 10, CSR reads monitored (regions: labels 0, row_ptr 1, col 2)."""
    torch, hr = env
    rp, col, mask = si.labelprop_graph(10, 8 * 1024, si.master_seed(2), 0.02)
    n = rp.shape[0] - 1
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    say("labelprop log, grouping", grouping)
    with hr.Context(access_log=True, wave_grouping=grouping) as ctx:
        r_lab, r_rp, r_col = ctx.shadow_alloc(label), ctx.shadow_alloc(rp_d), \
            ctx.shadow_alloc(col_d)
        assert (r_lab, r_rp, r_col) == (0, 1, 2)
        for L in range(2):
            ctx.labelprop_check(r_lab, label, rp_d, col_d, mask_d, tpb=256, r_row_ptr=r_rp,
                                r_col=r_col)
            ctx.kernel_end()
        recs, st = ctx.access_log()
        assert st == 0
    want = oracle.model_labelprop(rp, col, mask, 2, 256, monitor_csr=True)
    same(device_rows(recs, hr), oracle_rows(want))


PROGRAMS = [
    # seed, launches, blocks, threads, phases, max_ops, gwords, lwords, p_lds, wave width
    (1, 2, 4, 128, 4, 2, 64, 64, 0.3, 64),
    (5, 2, 33, 130, 5, 3, 300, 100, 0.5, 64),
    (8, 2, 6, 256, 4, 3, 2, 4, 0.2, 64),
    (12, 2, 5, 192, 5, 2, 128, 64, 0.4, 16),
]


@pytest.mark.parametrize("cfg", PROGRAMS, ids=lambda c: f"seed{c[0]}_b{c[2]}_t{c[3]}_w{c[9]}")
def test_program_access_log(env, cfg):
    torch, hr = env
    seed, launches, blocks, threads, phases, max_ops, gw, lw, p_lds, ww = cfg
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=3,
                             global_words=gw, lds_words=lw, p_lds=p_lds, wave_width=ww,
                             p_switch=0.05)
    want = oracle_rows(oracle.model_program(prog, ww))
    say("program log", cfg, len(want), "records")
    wb = int(ww).bit_length() - 1
    for kw in ({}, {"wave_grouping": True} if ww == 64 else {}):
        data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
        with hr.Context(access_log=True, wave_bits=wb, **kw) as ctx:
            regs = [ctx.shadow_alloc(d) for d in data]
            for launch in prog.launches:
                ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
                ctx.kernel_end()
            recs, st = ctx.access_log()
            assert st == 0
        same(device_rows(recs, hr, dict(zip(regs, range(len(regs))))), want)


def test_access_log_truncates_and_resets(env):
    torch, hr = env
    inp = torch.from_numpy(si.reduce_input(si.master_seed(0))).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    with hr.Context(access_log=True, log_capacity=1000) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out)
        recs, st = ctx.access_log()
        assert st == hr.HR_W_LOG_TRUNCATED and recs.shape[0] == 1000
        ctx.reset()
        recs, st = ctx.access_log()
        assert st == 0 and recs.shape[0] == 0
    with hr.Context() as ctx:
        with pytest.raises(hr.HRError):
            ctx.access_log()
