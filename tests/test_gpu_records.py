"""Race records on the GPU.  Which access completes a race depends on the
schedule, so each record is checked for validity against the oracle's access
log: its `before` and `with` summaries hold a pair of accesses at its key
that race by the pairwise definition, and `with` is the completing access
(thread, block, class).  Call-site ids match the workload, and a per-site
record limit keeps at most that many records per site, with a warning."""
import numpy as np
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


def check_records(recs, log, region_map, strict_with=True):
    keys = by_key(log)
    seen = set()
    for rec in recs:
        k = record_key(rec, region_map)
        assert k in keys, k
        why = record_problem(rec, keys[k], strict_with)
        assert why is None, (k, why, rec)
        seen.add(k)
    return seen


PROGRAMS = [
    # seed, launches, blocks, threads, phases, max_ops, gwords, lwords
    (21, 2, 4, 128, 4, 2, 64, 64),
    (22, 3, 8, 256, 5, 3, 256, 128),
    (23, 2, 6, 256, 4, 3, 2, 4),
]


@pytest.mark.parametrize("grouping", [False, True])
@pytest.mark.parametrize("cfg", PROGRAMS, ids=lambda c: f"seed{c[0]}")
def test_program_records_name_racing_pairs(env, cfg, grouping):
    torch, hr = env
    seed, launches, blocks, threads, phases, max_ops, gw, lw = cfg
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=3,
                             global_words=gw, lds_words=lw, p_lds=0.3)
    log = oracle.model_program(prog)
    want = oracle.flagged(log.copy())
    say("program records", cfg, "grouping", grouping, "oracle flags", len(want))
    data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    with hr.Context(wave_grouping=grouping) as ctx:
        regs = [ctx.shadow_alloc(d) for d in data]
        for launch in prog.launches:
            ctx.program_check(hr.DeviceProgram(launch), regs, prog.lds_words)
            ctx.kernel_end()
        recs, st = ctx.report()
    assert st == 0
    seen = check_records(recs, log, {r: i for i, r in enumerate(regs)},
                         strict_with=not grouping)
    assert seen == want and len(recs) == len(want)
    assert all(1 <= int(r["site"]) <= phases for r in recs)       # site = phase + 1


def test_jacobi_records_and_sites(env):
    torch, hr = env
    ny, nx, launches = 64, 80, 3
    seeds = si.jacobi_seeds(ny, nx, 5, count=6)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("jacobi records")
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 2)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    with hr.Context() as ctx:
        regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]
        tab_d = torch.from_numpy(tab).cuda()
        for L in range(launches):
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], tab_d)
            ctx.kernel_end()
        recs, st = ctx.report()
    assert st == 0
    log = oracle.model_jacobi(ny, nx, launches, tab)
    seen = check_records(recs, log, {regs[0]: 0, regs[1]: 1})
    assert seen == cf.jacobi_flagged(ny, nx, launches, seeds)
    assert {int(r["site"]) for r in recs} <= {hr.HR_SITE_JACOBI_OUT, hr.HR_SITE_JACOBI_SEED}
    assert all(int(r["kind"]) == hr.HR_WRITE for r in recs)


@pytest.mark.parametrize("drop", [0, 3, 8])
def test_reduce_records_and_sites(env, drop):
    torch, hr = env
    say("reduce records drop", drop)
    x = si.reduce_input(si.master_seed(0) + drop)
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    with hr.Context() as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out, drop=drop)
        ctx.kernel_end()
        recs, st = ctx.report()
    assert st == 0
    log = oracle.model_reduce(drop)
    seen = check_records(recs, log, {r_in: 0, r_out: 1})
    assert seen == cf.reduce_flagged(drop)
    lds_sites = {hr.HR_SITE_REDUCE_LEFT, hr.HR_SITE_REDUCE_RIGHT, hr.HR_SITE_REDUCE_SUM,
                 hr.HR_SITE_REDUCE_TOTAL}
    assert {int(r["site"]) for r in recs} <= lds_sites


def test_site_limit_caps_records_and_warns(env):
    """A per-site record limit drops records, never flagged locations: the
    report recovers the global races whose records were dropped from their
    sticky race words, also with 4-byte words, whose race words must then
    survive the launch-boundary clears."""
    torch, hr = env
    ny, nx, launches = 96, 96, 2
    seeds = si.jacobi_seeds(ny, nx, 9, count=12)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, launches, seeds)
    assert all(k[0] == 0 for k in want)
    say("site limit")
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 3)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = torch.from_numpy(tab).cuda()
    for word4 in (False, True):
        for limit in (0, 3, 1):
            say("  word4", word4, "limit", limit)
            with hr.Context(site_limit=limit, word4=word4) as ctx:
                regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]
                for L in range(launches):
                    ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2],
                                     tab_d)
                    ctx.kernel_end()
                recs, st = ctx.report()
                keys = ctx.flagged()
            remap = {regs[0]: 0, regs[1]: 1}
            assert {(0, remap[int(r["region"])], 0, int(r["index"])) for r in recs} == want
            if limit == 0:
                assert st == 0 and keys == want
                continue
            assert st & hr.HR_W_REPORT_LIMITED
            ring = recs[(recs["flags"] & hr.HR_RACE_SCANNED) == 0]
            per_site = {}
            for r in ring:
                per_site[int(r["site"])] = per_site.get(int(r["site"]), 0) + 1
            assert max(per_site.values()) <= limit and len(ring) < len(want)
