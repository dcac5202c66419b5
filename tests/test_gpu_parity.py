"""GPU parity: the HIP checker's flagged (space, region, block-if-LDS, index)
set must equal the oracle's, bit for bit, on the same seeded inputs.  The
work is integer and exact, so the tolerance is zero.  Calls go through the
C ABI (ctypes binding of libhr.so)."""
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


# ------------------------------------------------------------ reduction
@pytest.mark.parametrize("drop", [-1] + list(range(9)))
def test_reduce_flagged_set(env, drop):
    torch, hr = env
    say("reduce drop", drop)
    x = si.reduce_input(si.master_seed(0) + drop)
    inp = torch.from_numpy(x).cuda()
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    with hr.Context(count_checks=True) as ctx:
        r_in, r_out = ctx.shadow_alloc(inp), ctx.shadow_alloc(out)
        ctx.reduce_check(r_in, r_out, inp, out, drop=drop)
        ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status == 0
        assert ctx.check_count() == 3069
    log = oracle.model_reduce(drop)
    assert got == oracle.flagged(log) == cf.reduce_flagged(drop)
    if drop < 0:
        assert (out.cpu().numpy() == x.astype(np.int64).sum()).all()
        out2 = torch.zeros_like(out)
        hr.reduce_plain(inp, out2, -1)
        torch.cuda.synchronize()
        assert torch.equal(out, out2)


# ------------------------------------------------------- access programs
PROGRAMS = [
    # seed, launches, blocks, threads, phases, max_ops, gwords, lwords, p_lds
    (1, 2, 4, 128, 4, 2, 64, 64, 0.3),
    (2, 3, 16, 256, 5, 3, 512, 256, 0.4),
    (3, 2, 64, 256, 6, 2, 4096, 1024, 0.3),
    (4, 2, 8, 1000, 4, 2, 2048, 512, 0.3),
    (5, 2, 33, 130, 5, 3, 300, 100, 0.5),
    (6, 4, 3, 1024, 3, 1, 1024, 2048, 0.2),
    (7, 1, 200, 64, 8, 2, 8192, 64, 0.3),
    (8, 2, 6, 256, 4, 3, 2, 4, 0.2),           # heavy same-word contention
]


def run_program(torch, hr, prog, block_perm_seed=None, ctx_kwargs=None, tile=None, cols=13):
    """tile: give every global region a tiled shadow map, the region viewed as
    a 2-D array `cols` elements wide (rounded up to whole rows)."""
    if tile is None:
        data = [torch.zeros(w, dtype=torch.int32, device="cuda") for w in prog.global_words]
    else:
        data = [torch.zeros(((w + cols - 1) // cols, cols), dtype=torch.int32, device="cuda")
                for w in prog.global_words]
    with hr.Context(**(ctx_kwargs or {})) as ctx:
        regs = [ctx.shadow_alloc(d, tile=tile) for d in data]
        for launch in prog.launches:
            dp = hr.DeviceProgram(launch)
            bmap = None
            if block_perm_seed is not None:
                perm = np.random.default_rng(block_perm_seed).permutation(launch.blocks)
                bmap = torch.from_numpy(perm.astype(np.int32)).cuda()
            ctx.program_check(dp, regs, prog.lds_words, block_map=bmap)
            ctx.kernel_end()
        got = ctx.flagged()
        return got, ctx.status


@pytest.mark.parametrize("cfg", PROGRAMS, ids=lambda c: f"seed{c[0]}_b{c[2]}_t{c[3]}")
def test_program_flagged_set(env, cfg):
    torch, hr = env
    seed, launches, blocks, threads, phases, max_ops, gw, lw, p_lds = cfg
    prog = si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=3,
                             global_words=gw, lds_words=lw, p_lds=p_lds)
    want = oracle.flagged_program(prog)
    say("program", cfg, "oracle flags", len(want))
    got, st = run_program(torch, hr, prog)
    assert st == 0
    assert got == want
    # a different mapping of logical blocks to hardware blocks changes the
    # schedule but not the verdict
    got2, _ = run_program(torch, hr, prog, block_perm_seed=seed)
    assert got2 == want
    # wave grouping of same-word lanes changes the number of atomics only
    got3, st3 = run_program(torch, hr, prog, ctx_kwargs={"wave_grouping": True})
    assert st3 == 0 and got3 == want
    # so does a tiled address-to-shadow map (ragged rows of 13 elements)
    got4, st4 = run_program(torch, hr, prog, tile=(2, 1))
    assert st4 == 0 and got4 == want


@pytest.mark.parametrize("tile,cols", [((2, 2), 16), ((3, 1), 7), ((1, 3), 100), ((4, 4), 33),
                                       ((0, 2), 5)])
def test_program_tiled_shadow_map(env, tile, cols):
    """The generic hook's index-to-shadow map (a division by the row width)
    on ragged tiles, with and without wave grouping: the verdict is the
    oracle's, which knows nothing of shadow layouts."""
    torch, hr = env
    prog = si.random_program(31, launches=2, blocks=12, threads=256, phases=5, max_ops=3,
                             global_regions=3, global_words=700, lds_words=128, p_lds=0.3)
    want = oracle.flagged_program(prog)
    assert len(want) > 0
    say("program tiled map", tile, cols)
    got, st = run_program(torch, hr, prog, tile=tile, cols=cols)
    assert st == 0 and got == want
    got2, st2 = run_program(torch, hr, prog, tile=tile, cols=cols,
                            ctx_kwargs={"wave_grouping": True})
    assert st2 == 0 and got2 == want


def test_program_race_free_variants(env):
    torch, hr = env
    for kinds in [(1.0, 0.0, 0.0), (0.0, 0.0, 1.0)]:
        prog = si.random_program(17, launches=2, blocks=32, threads=256, phases=4,
                                 max_ops=3, global_regions=2, global_words=128,
                                 lds_words=64, kind_p=kinds)
        say("race-free program", kinds)
        got, st = run_program(torch, hr, prog)
        assert got == set() and st == 0


def test_program_empty_and_idle(env):
    torch, hr = env
    say("empty program")
    prog = si.random_program(3, launches=2, blocks=5, threads=70, phases=3, max_ops=0)
    got, st = run_program(torch, hr, prog)
    assert got == set() and st == 0


# --------------------------------------------------------------- Jacobi
JACOBI = [(64, 64, 3, 6), (50, 37, 2, 5), (33, 80, 4, 8), (96, 17, 3, 4), (16, 16, 2, 0),
          (256, 192, 3, 20),
          # degenerate shapes: one cell, one row, one column, one past a tile
          (1, 1, 2, 0), (2, 2, 3, 0), (1, 40, 3, 2), (40, 1, 3, 2), (1, 17, 2, 1), (17, 17, 3, 2),
          (15, 33, 2, 1)]


# Shadow maps of the stencil's grids: row-major, tiles of 4 x 4, 8 x 2 and
# 2 x 8 elements (one 128-byte line of 8-byte words per tile) and of 4 x 2
# (the kernels with a constant map: row-major, 4 x 4, 8 x 2, 4 x 2; the
# others read the map at run time).
TILES = [None, (2, 2), (3, 1), (1, 3), (2, 1)]


def tile_id(t):
    return "rowmajor" if t is None else f"tile{1 << t[0]}x{1 << t[1]}"


def run_jacobi(torch, hr, ny, nx, launches, tab, ctx_kwargs=None, grid_seed=1, tile=None):
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, grid_seed)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = None if tab is None else torch.from_numpy(tab).cuda()
    with hr.Context(**(ctx_kwargs or {})) as ctx:
        regs = [ctx.shadow_alloc(u[0], tile=tile), ctx.shadow_alloc(u[1], tile=tile)]
        for L in range(launches):
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2], tab_d)
            ctx.kernel_end()
        got = ctx.flagged()
        st = ctx.status
        count = ctx.check_count() if ctx_kwargs and ctx_kwargs.get("count_checks") else None
    return got, st, u, count


@pytest.mark.parametrize("tile", TILES, ids=tile_id)
@pytest.mark.parametrize("ny,nx,launches,count", JACOBI)
def test_jacobi_flagged_set(env, ny, nx, launches, count, tile):
    torch, hr = env
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + nx, count=count)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("jacobi", ny, nx, launches, count, tile_id(tile))
    got, st, _, n = run_jacobi(torch, hr, ny, nx, launches, tab, {"count_checks": True},
                               tile=tile)
    log = oracle.model_jacobi(ny, nx, launches, tab)
    assert st == 0
    assert n == log.shape[0]
    assert got == oracle.flagged(log) == cf.jacobi_flagged(ny, nx, launches, seeds)


def test_jacobi_race_free_output_matches_plain(env):
    torch, hr = env
    ny, nx = 200, 130
    say("jacobi race-free vs plain", ny, nx)
    got, st, u, _ = run_jacobi(torch, hr, ny, nx, 3, None)
    assert got == set() and st == 0
    p = [torch.from_numpy(si.jacobi_grid(ny, nx, 1)).cuda(), torch.zeros_like(u[1])]
    for L in range(3):
        hr.jacobi_plain(p[L % 2], p[(L + 1) % 2], None)
    torch.cuda.synchronize()
    assert torch.equal(u[1], p[1]) and torch.equal(u[0], p[0])


# ------------------------------------------------------- label propagation
@pytest.mark.parametrize("grouping", [False, True])
@pytest.mark.parametrize("scale,edges,p,tpb", [(10, 8 * 1024, 0.01, 256), (12, 8 * 4096, 0.02, 256),
                                               (13, 8 * 8192, 0.01, 128), (9, 4096, 0.05, 1000)])
def test_labelprop_flagged_set(env, scale, edges, p, tpb, grouping):
    torch, hr = env
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2) + scale, p)
    n = rp.shape[0] - 1
    say("labelprop", scale, edges, p, tpb, "grouping", grouping)
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    with hr.Context(count_checks=True, wave_grouping=grouping) as ctx:
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


def _lp_case(name):
    """Degenerate graphs: (row_ptr, col, mask) and the vertex count."""
    n = 70
    if name == "one_vertex":
        return [0, 0], [], []
    if name == "no_edges":
        return [0] * (n + 1), [], []
    if name == "self_loops_seeded":        # no other thread touches label[v]
        return list(range(n + 1)), list(range(n)), [1] * n
    if name == "star_out_seeded":          # vertex 0 writes every other label
        return [0] + [n - 1] * n, list(range(1, n)), [1] * (n - 1)
    if name == "star_in_seeded":           # every vertex writes label[0]
        return [0] + list(range(n)), [0] * (n - 1), [1] * (n - 1)
    if name == "star_in_atomic":           # the same with atomics only
        return [0] + list(range(n)), [0] * (n - 1), [0] * (n - 1)
    raise ValueError(name)


@pytest.mark.parametrize("name", ["one_vertex", "no_edges", "self_loops_seeded", "star_out_seeded",
                                  "star_in_seeded", "star_in_atomic"])
@pytest.mark.parametrize("tpb", [1, 64, 1024])
def test_labelprop_degenerate_graphs(env, name, tpb):
    torch, hr = env
    rp, col, mask = (np.asarray(x, dtype=t) for x, t in zip(_lp_case(name),
                                                           (np.int32, np.int32, np.uint8)))
    n = rp.shape[0] - 1
    say("labelprop degenerate", name, "tpb", tpb)
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    rp_d = torch.from_numpy(rp).cuda()
    # an edge-free graph still hands the kernel some col / mask buffer
    col_d = torch.from_numpy(col if col.size else np.zeros(1, np.int32)).cuda()
    mask_d = torch.from_numpy(mask if mask.size else np.zeros(1, np.uint8)).cuda()
    with hr.Context(count_checks=True) as ctx:
        r_lab = ctx.shadow_alloc(label)
        for L in range(2):
            ctx.labelprop_check(r_lab, label, rp_d, col_d, mask_d, tpb=tpb)
            ctx.kernel_end()
        got = ctx.flagged()
        cnt = ctx.check_count()
        assert ctx.status == 0
    log = oracle.model_labelprop(rp, col, mask, 2, tpb)
    assert cnt == log.shape[0]
    assert got == oracle.flagged(log) == cf.labelprop_flagged(rp, col, mask)


# ----------------------------------------------------- failure handling
def test_clock_overflow_stops_with_warning(env):
    """bc_bits=2 allows 3 block barriers; a 6-barrier program overflows.  The
    warning is set and races seen before the overflow are still reported."""
    torch, hr = env
    G = si.SPACE_GLOBAL
    per = [[[[] for _ in range(64)] for _ in range(2)] for _ in range(6)]
    per[0][0][0].append(si.op_word(G, 0, si.KIND_W, 3))
    per[0][1][0].append(si.op_word(G, 0, si.KIND_W, 3))       # race, epoch 0
    per[5][0][0].append(si.op_word(G, 0, si.KIND_W, 5))
    per[5][1][0].append(si.op_word(G, 0, si.KIND_W, 5))       # race after overflow
    launch = si.build_launch(2, 64, [2] * 6, [0] * 6, per)
    prog = si.Program([launch], [16], 16)
    say("clock overflow")
    got, st = run_program(torch, hr, prog, ctx_kwargs={"bc_bits": 2})
    assert st & hr.HR_W_CLOCK_OVERFLOW
    assert got == {(0, 0, 0, 3)}
    got, st = run_program(torch, hr, prog)
    assert st == 0 and got == {(0, 0, 0, 3), (0, 0, 0, 5)}


def test_ring_overflow_recovers_global_set(env):
    torch, hr = env
    prog = si.random_program(23, launches=2, blocks=16, threads=256, phases=3, max_ops=2,
                             global_regions=2, global_words=256, lds_words=64, p_lds=0.3)
    want = oracle.flagged_program(prog)
    want_global = {k for k in want if k[0] == 0}
    assert len(want) > 4
    say("ring overflow")
    got, st = run_program(torch, hr, prog, ctx_kwargs={"ring_capacity": 1})
    assert st & hr.HR_W_RING_OVERFLOW
    assert {k for k in got if k[0] == 0} == want_global
    assert got <= want


def test_out_of_range_operation_is_skipped(env):
    torch, hr = env
    G = si.SPACE_GLOBAL
    per = [[[[si.op_word(G, 0, si.KIND_W, 100)], [si.op_word(1, 0, si.KIND_W, 50)]]]]
    launch = si.build_launch(1, 2, [0], [0], per)
    prog = si.Program([launch], [16], 16)
    say("out of range")
    got, st = run_program(torch, hr, prog)
    assert st & hr.HR_W_OUT_OF_RANGE and got == set()


def test_shadow_budget_and_bad_arguments(env):
    torch, hr = env
    say("budget")
    x = torch.zeros(1024, dtype=torch.int32, device="cuda")
    with hr.Context(shadow_budget=4096) as ctx:
        with pytest.raises(hr.HRError) as e:
            ctx.shadow_alloc(x)
        assert e.value.status == hr.HR_E_NOMEM
    with hr.Context() as ctx:
        r = ctx.shadow_alloc(x)
        y = torch.zeros(256, dtype=torch.int32, device="cuda")
        with pytest.raises(hr.HRError):          # region too small for 512 inputs
            ctx.reduce_check(r, r, y, y, -1)
    say("labelprop argument checks")
    with hr.Context() as ctx:
        lab = torch.zeros(64, dtype=torch.int32, device="cuda")
        rp = torch.zeros(65, dtype=torch.int32, device="cuda")
        r_lab = ctx.shadow_alloc(lab)

        def raw(ptrs, tpb):          # the C entry point itself, without the binding's checks
            return hr._lib.hr_labelprop_check(ctx._c, r_lab, hr.NO_REGION, hr.NO_REGION,
                                              *ptrs, 64, tpb, None)
        for bad in ((0, 1, 1, 1), (1, 0, 1, 1), (1, 1, 0, 1), (1, 1, 1, 0)):
            ptrs = [t.data_ptr() if ok else None for t, ok in zip((lab, rp, rp, rp), bad)]
            assert raw(ptrs, 64) == hr.HR_E_INVAL, bad
        good = [lab.data_ptr(), rp.data_ptr(), rp.data_ptr(), rp.data_ptr()]
        assert raw(good, 2048) == hr.HR_E_INVAL     # more than 1024 threads per block
        assert raw(good, 0) == hr.HR_E_INVAL


def test_launch_epoch_wrap(env):
    """More than 512 launches: the shadow is cleared when the 9-bit launch
    epoch wraps; the flagged set is unchanged."""
    torch, hr = env
    ny, nx = 48, 48
    seeds = si.jacobi_seeds(ny, nx, 77, count=2)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("epoch wrap")
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 530, tab)
    assert st == 0
    assert got == cf.jacobi_flagged(ny, nx, 530, seeds)
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 530, None)
    assert got == set()


@pytest.mark.parametrize("tile", TILES[1:], ids=tile_id)
def test_ring_overflow_tiled_map(env, tile):
    """With a ring of one record the global set comes back from the race
    words, whose tiled offsets (ragged edge tiles included) map back to
    element indices."""
    torch, hr = env
    ny, nx = 70, 45
    seeds = si.jacobi_seeds(ny, nx, 91, count=6)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, 3, seeds)
    assert len(want) > 1
    say("ring overflow, tiled map", tile_id(tile))
    got, st, _, _ = run_jacobi(torch, hr, ny, nx, 3, tab, {"ring_capacity": 1}, tile=tile)
    assert st & hr.HR_W_RING_OVERFLOW
    assert got == want == oracle.flagged(oracle.model_jacobi(ny, nx, 3, tab))


def test_tiled_map_argument_checks(env):
    torch, hr = env
    u = torch.zeros((40, 24), dtype=torch.float32, device="cuda")
    v = torch.zeros((40, 24), dtype=torch.float32, device="cuda")
    with hr.Context() as ctx:
        with pytest.raises(hr.HRError):
            ctx.shadow_alloc(u, tile=(5, 0))           # a tile side above 16
        # a tiled map whose rows are not the stencil's rows is refused
        r0 = ctx.shadow_alloc(u.view(24, 40), tile=(2, 2))
        r1 = ctx.shadow_alloc(v, tile=(2, 2))
        with pytest.raises(hr.HRError):
            ctx.jacobi_check(r0, r1, u, v, None)


def test_ring_overflow_across_epoch_wrap(env):
    """Races seen only before the launch epoch wraps, with a ring that holds
    one record: the clear at the wrap must not lose the global races that
    only their race words still hold."""
    torch, hr = env
    ny, nx = 48, 48
    seeds = si.jacobi_seeds(ny, nx, 78, count=3)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    want = cf.jacobi_flagged(ny, nx, 4, seeds)
    assert len(want) > 1 and all(k[0] == 0 for k in want)
    say("ring overflow across epoch wrap")
    u = [torch.from_numpy(si.jacobi_grid(ny, nx, 1)).cuda(),
         torch.zeros((ny, nx), dtype=torch.float32, device="cuda")]
    tab_d = torch.from_numpy(tab).cuda()
    with hr.Context(ring_capacity=1) as ctx:
        regs = [ctx.shadow_alloc(u[0]), ctx.shadow_alloc(u[1])]
        for L in range(530):                       # seeded only in the first 4 launches
            ctx.jacobi_check(regs[L % 2], regs[(L + 1) % 2], u[L % 2], u[(L + 1) % 2],
                             tab_d if L < 4 else None)
            ctx.kernel_end()
        got = ctx.flagged()
        assert ctx.status & hr.HR_W_RING_OVERFLOW
    assert got == want


# ------------------------------------------------------------- full size
def golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("tile", TILES, ids=tile_id)
def test_jacobi_full_size(env, tile):
    """4096 x 4096, 16 x 16 blocks, 20 launches, 66 seeded blocks: the flagged
    set equals the oracle's on the whole job's access log (streamed by
    oracle/goldens.py into tests/golden/), and the device access count equals
    the number of records the oracle checked; under every shadow map."""
    torch, hr = env
    ny = nx = 4096
    launches = 20
    gold = golden("jacobi_4096x4096_20launches.json")
    want = {tuple(k) for k in gold["keys"]}
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1))
    tab = si.jacobi_seed_table(ny, nx, seeds)
    say("jacobi full size", ny, nx, launches, len(seeds), tile_id(tile))
    got, st, _, n = run_jacobi(torch, hr, ny, nx, launches, tab, {"count_checks": True},
                               grid_seed=si.master_seed(1), tile=tile)
    assert st == 0
    assert got == want and len(want) == gold["flagged"]
    assert n == gold["checks"]


def test_labelprop_full_size(env):
    """R-MAT scale 22, 2^25 edges, 1 % seeded edges, 10 launches: the flagged
    set equals the oracle's on the whole job's access log (its size and
    SHA-256 in tests/golden/), with a ring that holds every record and with
    one that overflows (the set then comes from the race-word scan)."""
    torch, hr = env
    from oracle.goldens import key_digest
    gold = golden("labelprop_rmat22_10launches.json")
    scale, edges, launches = 22, 1 << 25, 10
    say("labelprop full size: building graph")
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2), 0.01)
    n = 1 << scale
    label = torch.arange(n, dtype=torch.int32, device="cuda")
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    mask_d = torch.from_numpy(mask).cuda()
    say("labelprop full size: running,", gold["flagged"], "racy vertices expected")
    for ring, expect_overflow in ((1 << 21, False), (65536, True)):
        label.copy_(torch.arange(n, dtype=torch.int32, device="cuda"))
        with hr.Context(ring_capacity=ring, count_checks=True) as ctx:
            r_lab = ctx.shadow_alloc(label)
            for L in range(launches):
                ctx.labelprop_check(r_lab, label, rp_d, col_d, mask_d, tpb=256)
                ctx.kernel_end()
            got = ctx.flagged()
            assert bool(ctx.status & hr.HR_W_RING_OVERFLOW) == expect_overflow
            assert ctx.status & ~hr.HR_W_RING_OVERFLOW == 0
            assert ctx.check_count() == gold["checks"]
        ks = sorted(got)
        assert len(got) == gold["flagged"] and key_digest(got) == gold["sha256"]
        assert [list(k) for k in ks[:16]] == gold["first_keys"]


def _sparse_launch(blocks, threads, scopes, entries):
    """A launch of `blocks` x `threads` in which only the (phase, block,
    thread) keys of `entries` have operations (op lists)."""
    n = len(scopes) * blocks * threads
    counts = np.zeros(n, dtype=np.int64)
    idx = {(p * blocks + b) * threads + t: ops for (p, b, t), ops in entries.items()}
    for i, ops in idx.items():
        counts[i] = len(ops)
    op_off = np.zeros(n + 1, dtype=np.int32)
    op_off[1:] = np.cumsum(counts)
    flat = np.zeros(int(op_off[-1]), dtype=np.uint32)
    for i, ops in idx.items():
        flat[op_off[i]:op_off[i] + len(ops)] = ops
    return si.Launch(blocks, threads, np.asarray(scopes, np.uint8),
                     np.zeros(len(scopes), np.uint64), op_off, flat)


@pytest.mark.parametrize("table", [False, True])
def test_program_largest_block_ids(env, table):
    """2^22 - 1 logical blocks, the most a launch may have: accessors whose
    block ids differ only in the top bits of the 22-bit field (1 and
    2^21 + 1) race, the last block's LDS race carries its id, and ordered
    or atomic accesses of far-apart blocks stay clean -- the oracle's set."""
    torch, hr = env
    B = (1 << 22) - 1
    G, L, R, W, A = si.SPACE_GLOBAL, si.SPACE_LDS, si.KIND_R, si.KIND_W, si.KIND_A
    op = si.op_word
    entries = {
        (0, 0, 0): [op(G, 0, W, 0)], (0, B - 1, 1): [op(G, 0, R, 0)],           # race
        (0, 1, 0): [op(G, 0, W, 2)], (0, (1 << 21) + 1, 0): [op(G, 0, W, 2)],   # race
        (0, 1 << 21, 0): [op(G, 0, W, 1)], (1, 1 << 21, 1): [op(G, 0, R, 1)],   # ordered
        (0, B - 1, 0): [op(G, 0, W, 3)], (1, B - 1, 1): [op(G, 0, W, 3)],       # ordered
        (0, 2, 0): [op(G, 0, A, 4)], (0, B - 2, 1): [op(G, 0, A, 4)],           # atomics
        (1, B - 1, 0): [op(L, 0, W, 0)],                                          # LDS race
    }
    entries[(1, B - 1, 1)] = entries[(1, B - 1, 1)] + [op(L, 0, W, 0)]
    launch = _sparse_launch(B, 2, [si.SCOPE_BLOCK, si.SCOPE_NONE], entries)
    prog = si.Program([launch], [8], 2)
    want = oracle.flagged_program(prog)
    assert want == {(0, 0, 0, 0), (0, 0, 0, 2), (1, 0, B - 1, 0)}
    say("largest block ids, table", table)
    data = torch.zeros(8, dtype=torch.int32, device="cuda")
    with hr.Context(fsm_table=table) as ctx:
        reg = ctx.shadow_alloc(data)
        ctx.program_check(hr.DeviceProgram(launch), [reg], 2)
        ctx.kernel_end()
        got, st = ctx.flagged(), ctx.status
    assert st == 0
    assert {(sp, 0 if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in got} == want
    with hr.Context() as ctx:                  # one block more than the field holds
        reg = ctx.shadow_alloc(data)
        big = _sparse_launch(B + 1, 1, [si.SCOPE_NONE], {})
        with pytest.raises(hr.HRError):
            ctx.program_check(hr.DeviceProgram(big), [reg], 2)


def test_program_largest_threads_and_nested_block_ids(env):
    """1024-thread blocks (16 waves): lanes of the first and last wave race,
    a wave barrier in the last wave orders its own lanes only; and with
    tiles nested in waves, 2^20 blocks, the most the nested words hold (ids
    below 2^20): block ids that differ only in the top bit of their 20-bit
    field race.
    Each set is the oracle's."""
    torch, hr = env
    G, L, R, W = si.SPACE_GLOBAL, si.SPACE_LDS, si.KIND_R, si.KIND_W
    op = si.op_word
    entries = {
        (0, 1, 0): [op(G, 0, W, 0)], (0, 1, 1023): [op(G, 0, R, 0)],        # race
        (0, 0, 960): [op(L, 0, W, 5)], (1, 0, 1023): [op(L, 0, R, 5)],      # wave 15: ordered
        (0, 0, 959): [op(L, 0, W, 6)], (1, 0, 1022): [op(L, 0, R, 6)],      # waves 14, 15: race
    }
    launch = _sparse_launch(2, 1024, [si.SCOPE_WAVE, si.SCOPE_NONE], entries)
    launch.wave_mask[0] = 1 << 15                                            # only wave 15 syncs
    prog = si.Program([launch], [8], 8)
    want = oracle.flagged_program(prog)
    assert want == {(0, 0, 0, 0), (1, 0, 0, 6)}
    data = torch.zeros(8, dtype=torch.int32, device="cuda")
    say("1024-thread blocks")
    with hr.Context() as ctx:
        reg = ctx.shadow_alloc(data)
        ctx.program_check(hr.DeviceProgram(launch), [reg], 8)
        ctx.kernel_end()
        got, st = ctx.flagged(), ctx.status
    assert st == 0 and {(sp, 0 if sp == 0 else rg, lb, ix) for sp, rg, lb, ix in got} == want

    B = 1 << 20
    entries = {(0, 1, 0): [op(G, 0, W, 1)], (0, (1 << 19) + 1, 1): [op(G, 0, W, 1)],   # race
               (0, B - 1, 0): [op(G, 0, W, 2)], (1, B - 1, 1): [op(G, 0, R, 2)]}    # tile-ordered
    launch = _sparse_launch(B, 2, [si.SCOPE_TILE, si.SCOPE_NONE], entries)
    launch.wave_mask[0] = 1                                                  # tile 0 syncs
    prog = si.Program([launch], [8], 2)
    want = oracle.flagged_program(prog, 64, 2)
    assert want == {(0, 0, 0, 1)}
    say("nested, 2^20 blocks")
    with hr.Context(nested_tiles=True, wave_bits=1) as ctx:
        reg = ctx.shadow_alloc(data)
        ctx.program_check(hr.DeviceProgram(launch), [reg], 2)
        ctx.kernel_end()
        got, st = ctx.flagged(), ctx.status
        assert st == 0 and {(sp, 0, lb, ix) for sp, rg, lb, ix in got} == want
        with pytest.raises(hr.HRError):        # one block more than the nested field holds
            ctx.program_check(hr.DeviceProgram(_sparse_launch(B + 1, 1, [si.SCOPE_NONE], {})),
                              [reg], 2)
