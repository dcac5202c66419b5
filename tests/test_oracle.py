"""Pins of the race oracle against what the paper and the mathematics fix:
the paper's litmus kernels, an independent schedule brute force, closed-form
flagged sets of the workloads, invariants, and planted mistakes that the pins
must catch."""
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle import brute
from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- listings
def listing_program(case):
    blocks, threads = case["blocks"], case["threads"]
    G = si.SPACE_GLOBAL
    R, W = si.KIND_R, si.KIND_W
    if case["kernel"] == "race_noSync":
        # val = data[0]; data[0] = i + val;
        ops = [[[[si.op_word(G, 0, R, 0), si.op_word(G, 0, W, 0)]
                 for t in range(threads)] for b in range(blocks)]]
        scopes, masks = [0], [0]
    elif case["kernel"] == "race_blockSync":
        # val = data[0]; __syncthreads(); if (tid > 0) data[tid-1] = tid;
        p0 = [[[si.op_word(G, 0, R, 0)] for t in range(threads)] for b in range(blocks)]
        p1 = [[([si.op_word(G, 0, W, t - 1)] if t > 0 else []) for t in range(threads)]
              for b in range(blocks)]
        ops, scopes, masks = [p0, p1], [si.SCOPE_BLOCK, 0], [0, 0]
    elif case["kernel"] == "multiRead_Race":
        n = case["len"]
        # if (tid < len-2) { s = data[tid]; s += data[tid+1]; data[tid+1] = s; }
        p0 = [[([si.op_word(G, 0, R, t), si.op_word(G, 0, R, t + 1),
                 si.op_word(G, 0, W, t + 1)] if t < n - 2 else [])
               for t in range(threads)] for b in range(blocks)]
        ops, scopes, masks = [p0], [0], [0]
    else:
        raise ValueError(case["kernel"])
    launch = si.build_launch(blocks, threads, scopes, masks, ops)
    return si.Program(launches=[launch], global_words=[64], lds_words=0)


def golden_cases():
    with open(os.path.join(GOLDEN, "listings.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c["name"])
def test_listing_verdicts(case):
    prog = listing_program(case)
    want = {(0, 0, 0, i) for i in case["flagged"]}
    ww = case["wave_width"]
    assert oracle.flagged_program(prog, ww) == want
    assert brute.flagged_program(prog, ww) == want


# ------------------------------------------------------------- brute force
BRUTE_SETTINGS = [
    # blocks, threads, wave_width, phases, max_ops, gwords, lwords
    (1, 4, 2, 3, 2, 3, 2),
    (2, 2, 1, 3, 2, 3, 2),
    (2, 3, 2, 4, 1, 4, 3),
    (1, 3, 1, 4, 2, 2, 2),
    (2, 2, 2, 2, 3, 4, 2),
]


@pytest.mark.parametrize("setting", BRUTE_SETTINGS)
def test_oracle_equals_schedule_brute_force(setting):
    blocks, threads, ww, phases, max_ops, gw, lw = setting
    racy = clean = 0
    for s in range(60):
        prog = si.random_program(1000 * setting[0] + 37 * s + threads, launches=2,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=1, global_words=gw,
                                 lds_words=lw, kind_p=(0.6, 0.2, 0.2),
                                 scope_p=(0.2, 0.4, 0.4), wave_width=ww)
        a = oracle.flagged_program(prog, ww)
        b = brute.flagged_program(prog, ww)
        assert a == b, (setting, s)
        log = oracle.model_program(prog, ww)
        touched = {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
                   for r in log}
        racy += len(a)
        clean += len(touched - a)
    # the sample must hold both verdicts, or it pins nothing
    assert racy > 0 and clean > 0


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("drop", [-1] + list(range(9)))
def test_reduce_closed_form(drop):
    log = oracle.model_reduce(drop)
    assert log.shape[0] == 3069      # 512 + 512 + 3*511 + 256 + 256
    assert oracle.flagged(log) == cf.reduce_flagged(drop)


@pytest.mark.parametrize("n,threads,blocks", [(512, 256, 1), (256, 256, 3), (64, 128, 2),
                                             (2, 64, 1), (128, 64, 4), (2048, 1024, 2)])
def test_scaled_reduce_closed_form(n, threads, blocks):
    """The scaled reduction used by batched jobs; with n = 2 * threads there
    is no barrier after the loads, as in the paper-sized case."""
    steps = n.bit_length() - 1
    for drop in [-1] + list(range(steps)):
        log = oracle.model_reduce_n(n, threads, blocks, drop)
        assert log.shape[0] == blocks * (2 * n + 3 * (n - 1) + 2 * threads)
        assert oracle.flagged(log) == cf.reduce_n_flagged(n, threads, blocks, drop)
    if (n, threads, blocks) == (512, 256, 1):
        assert np.array_equal(oracle.model_reduce_n(512, 256, 1, 3), oracle.model_reduce(3))


@pytest.mark.parametrize("ny,nx,launches,count", [
    (64, 64, 3, 6), (50, 37, 2, 5), (33, 80, 4, 8), (16, 16, 2, 0), (96, 17, 3, 4)])
def test_jacobi_closed_form(ny, nx, launches, count):
    seeds = si.jacobi_seeds(ny, nx, si.master_seed(1) + ny, count=count)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    log = oracle.model_jacobi(ny, nx, launches, tab)
    assert oracle.flagged(log) == cf.jacobi_flagged(ny, nx, launches, seeds)
    assert oracle.flagged(oracle.model_jacobi(ny, nx, launches, None)) == set()


def test_jacobi_access_counts_full_size():
    """Per-launch access count of the 4096^2 sweep: 20,955,136 global reads,
    as many LDS writes, 83,869,696 LDS reads and 16,777,216 global writes."""
    lib = oracle._lib()
    n = lib.orc_model_jacobi(4096, 4096, 0, 1, None, 0, 256, 0, 256, None, 0)
    assert n == 20955136 * 2 + 83869696 + 16777216


def test_jacobi_window_is_exact_for_centre_block():
    ny = nx = 80
    seeds = si.jacobi_seeds(ny, nx, 99, count=10)
    tab = si.jacobi_seed_table(ny, nx, seeds)
    full = oracle.flagged(oracle.model_jacobi(ny, nx, 2, tab))
    nbx = 5
    for bx, by in [(2, 2), (1, 3), (0, 0), (4, 4)]:
        win = (max(bx - 1, 0), min(bx + 2, nbx), max(by - 1, 0), min(by + 2, nbx))
        got = oracle.flagged(oracle.model_jacobi(ny, nx, 2, tab, window=win))
        b = by * nbx + bx

        def owned(k):
            sp, rg, lb, ix = k
            if sp == 1:
                return lb == b
            y, x = divmod(ix, nx)
            return y // 16 == by and x // 16 == bx
        assert {k for k in got if owned(k)} == {k for k in full if owned(k)}


@pytest.mark.parametrize("scale,edges,p", [(10, 8 * 1024, 0.01), (12, 8 * 4096, 0.02),
                                          (8, 4096, 0.05)])
def test_labelprop_closed_form(scale, edges, p):
    rp, col, mask = si.labelprop_graph(scale, edges, si.master_seed(2) + scale, p)
    log = oracle.model_labelprop(rp, col, mask, 2, 256)
    assert oracle.flagged(log) == cf.labelprop_flagged(rp, col, mask)
    assert oracle.flagged(oracle.model_labelprop(rp, col, np.zeros_like(mask), 2)) == set()
    # monitoring the CSR arrays adds reads only: nothing new is flagged
    log = oracle.model_labelprop(rp, col, mask, 1, 256, monitor_csr=True)
    assert oracle.flagged(log) == cf.labelprop_flagged(rp, col, mask)


def test_labelprop_vertex_sample_is_exact():
    rp, col, mask = si.labelprop_graph(11, 8 * 2048, 5, 0.02)
    full = cf.labelprop_flagged(rp, col, mask)
    rng = np.random.default_rng(3)
    keep = (rng.random(2048) < 0.1).astype(np.uint8)
    keep[:8] = 1                          # the hubs
    got = oracle.flagged(oracle.model_labelprop(rp, col, mask, 1, 256, keep=keep))
    assert got == {k for k in full if keep[k[3]]}


def test_race_free_programs_flag_nothing():
    """Programs whose locations are each touched by one thread, or only read,
    or only accessed atomically, never race."""
    for s in range(20):
        prog = si.random_program(s, launches=2, blocks=3, threads=70, phases=3,
                                 max_ops=3, kind_p=(1.0, 0.0, 0.0))
        assert oracle.flagged_program(prog) == set()
        prog = si.random_program(s, launches=2, blocks=3, threads=70, phases=3,
                                 max_ops=3, kind_p=(0.0, 0.0, 1.0))
        assert oracle.flagged_program(prog) == set()


def test_every_injected_race_is_flagged():
    """A write injected into a race-free program races with a concurrent
    access of another thread to the same location."""
    rng = np.random.default_rng(11)
    for s in range(20):
        prog = si.random_program(s, launches=1, blocks=2, threads=130, phases=3,
                                 max_ops=2, kind_p=(1.0, 0.0, 0.0), p_lds=0.0,
                                 global_words=32)
        launch = prog.launches[0]
        # inject: thread t of block b writes location x in phase p, where some
        # other thread of another block reads x in the same launch
        reads = []
        for p in range(launch.phases):
            for b in range(launch.blocks):
                for t in range(launch.threads):
                    for w in launch.thread_ops(p, b, t):
                        reads.append((p, b, t, si.op_fields(w)[3]))
        p, b, t, x = reads[int(rng.integers(0, len(reads)))]
        other_b = 1 - b
        per = [[[list(launch.thread_ops(pp, bb, tt)) for tt in range(launch.threads)]
                for bb in range(launch.blocks)] for pp in range(launch.phases)]
        per[0][other_b][5].append(si.op_word(0, 0, si.KIND_W, x))
        new = si.build_launch(launch.blocks, launch.threads, launch.scope,
                              launch.wave_mask, per)
        p2 = si.Program(launches=[new], global_words=prog.global_words, lds_words=64)
        assert (0, 0, 0, x) in oracle.flagged_program(p2)


# -------------------------------------------------------- planted mistakes
MUTANTS = {
    "no_wave_barrier_order": (r"if \(p->wc != c->wc\) return 0;", ""),
    "no_block_barrier_order": (r"if \(p->bc != c->bc\) return 0;", ""),
    "no_launch_order": [(r"if \(p->launch != c->launch\) return 0;", ""),
                        (r"while \(b < k && recs\[b\]\.launch == recs\[a\]\.launch\) \+\+b;",
                         "while (b < k) ++b;")],
    "writes_do_not_conflict": (r"p->kind == c->kind && p->kind != K_WRITE", "p->kind == c->kind"),
    "atomics_conflict": [(r"p->kind == c->kind && p->kind != K_WRITE", "p->kind == c->kind && p->kind == K_READ"),
                         (r"if \(g\[i\]\.kind == K_WRITE\) scratch_w", "if (g[i].kind != K_READ) scratch_w")],
    "reads_conflict_with_reads": [(r"p->kind == c->kind && p->kind != K_WRITE", "0"),
                                  (r"if \(g\[i\]\.kind == K_WRITE\) scratch_w", "if (1) scratch_w")],
    "thread_id_without_block": (r"if \(p->block == c->block && p->thread == c->thread\) return 0;",
                                "if (p->thread == c->thread) return 0;"),
    "wave_barrier_orders_across_waves": (
        r"if \(p->thread / wave_width == c->thread / wave_width\) \{", "{"),
    # nested tiles (the tile level of the happens-before and of the model)
    "no_tile_barrier_order": (r"p->tc != c->tc\)\s*return 0;", "0) return 0;"),
    "tile_barrier_orders_across_tiles": (
        r"tile_width && p->thread / tile_width == c->thread / tile_width &&", "tile_width &&"),
    # (not restarting the tile epochs at a wave barrier is no mistake: with
    # equal wave epochs the tile clocks still differ exactly when a tile
    # barrier lies between, so the log's verdict cannot change)
    "tile_barrier_advances_every_tile": (
        r"scope\[p\] == 3 && tile_width && g < 64 && \(\(wave_mask\[p\] >> g\) & 1\)",
        "scope[p] == 3 && tile_width"),
    "reduce_model_drops_epilogue_read": (
        r"emit\(&s, SP_LDS, 0, 0, K_READ, launch, b, t, bc, 0\);", ""),
    "reduce_model_no_load_barrier": (r"if \(n != 2 \* T\) \+\+bc;", ""),
}


def _pins_hold():
    try:
        for case in golden_cases():
            prog = listing_program(case)
            if oracle.flagged_program(prog, case["wave_width"]) != {
                    (0, 0, 0, i) for i in case["flagged"]}:
                return False
        for drop in [-1, 3, 8]:
            if oracle.flagged(oracle.model_reduce(drop)) != cf.reduce_flagged(drop):
                return False
        for n, t, b, drop in [(64, 64, 2, 1), (128, 128, 1, -1), (32, 64, 2, 4)]:
            if oracle.flagged(oracle.model_reduce_n(n, t, b, drop)) != cf.reduce_n_flagged(n, t, b, drop):
                return False
        seeds = si.jacobi_seeds(64, 64, 5, count=6)
        tab = si.jacobi_seed_table(64, 64, seeds)
        if oracle.flagged(oracle.model_jacobi(64, 64, 3, tab)) != cf.jacobi_flagged(64, 64, 3, seeds):
            return False
        rp, col, mask = si.labelprop_graph(9, 4096, 7, 0.03)
        if oracle.flagged(oracle.model_labelprop(rp, col, mask, 2)) != cf.labelprop_flagged(rp, col, mask):
            return False
        for setting in BRUTE_SETTINGS[:3]:
            blocks, threads, ww, phases, max_ops, gw, lw = setting
            for s in range(25):
                prog = si.random_program(s, launches=2, blocks=blocks, threads=threads,
                                         phases=phases, max_ops=max_ops, global_regions=1,
                                         global_words=gw, lds_words=lw,
                                         kind_p=(0.6, 0.2, 0.2), wave_width=ww)
                if oracle.flagged_program(prog, ww) != brute.flagged_program(prog, ww):
                    return False
        for prog, want in nested_closed_cases():
            if oracle.flagged_program(prog, 64, 2) != want:
                return False
        for setting in NESTED_SETTINGS[:3]:
            for prog, tw in nested_programs(setting, 20):
                if oracle.flagged_program(prog, 64, tw) != brute.flagged_program(prog, 64, tw):
                    return False
        return True
    except AssertionError:
        return False


# Tiles nested in waves: blocks, threads (lanes of one wave), tile width,
# phases, max ops, global words, LDS words.
NESTED_SETTINGS = [
    (1, 4, 2, 3, 2, 2, 2),
    (1, 4, 2, 4, 1, 1, 1),
    (2, 2, 1, 3, 2, 2, 1),
    (1, 3, 1, 3, 2, 2, 2),
    (1, 6, 2, 3, 1, 2, 1),
]


def nested_programs(setting, n, base=0):
    """Random programs mixing block, wave and tile barriers (one wave per
    block, so every wave barrier spans the tiles of the block)."""
    blocks, threads, tw, phases, max_ops, gw, lw = setting
    for s in range(n):
        prog = si.random_program(base + 3 * s + threads, launches=2, blocks=blocks,
                                 threads=threads, phases=phases, max_ops=max_ops,
                                 global_regions=1, global_words=gw, lds_words=lw,
                                 kind_p=(0.6, 0.2, 0.2), scope_p=(0.25, 0.2, 0.15, 0.4),
                                 tile_width=tw)
        yield prog, tw


@pytest.mark.parametrize("setting", NESTED_SETTINGS)
def test_nested_tiles_oracle_equals_brute_force(setting):
    """Tiles nested in waves, each with their own barriers (tile epochs that a
    wave barrier restarts): the pairwise oracle equals the operational brute
    force, which knows only that a barrier waits for its whole group."""
    racy = clean = 0
    for prog, tw in nested_programs(setting, 40, base=100):
        want = brute.flagged_program(prog, 64, tw)
        assert oracle.flagged_program(prog, 64, tw) == want
        keys = {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
                for r in oracle.model_program(prog, 64, tw)}
        racy += len(want)
        clean += len(keys - want)
    assert racy > 0 and clean > 0


def nested_closed_cases():
    """(program, flagged set) pairs with two tiles of 2 lanes in one wave:
    lane 0 writes, then after a barrier (or none) lane 1 (same tile) or lane
    2 (the other tile) reads.  A tile barrier orders only its own tile's
    lanes, and only tiles in its mask advance; a wave barrier orders all."""
    G, W, R = si.SPACE_GLOBAL, si.KIND_W, si.KIND_R

    def prog(second, scope, mask):
        first = [[si.op_word(G, 0, W, 0)], [], [], []]
        return si.Program([si.build_launch(1, 4, [scope, 0], [mask, 0], [[first], [second]])],
                          [2], 2)
    r1 = [[], [si.op_word(G, 0, R, 0)], [], []]         # lane 1: same tile as lane 0
    r2 = [[], [], [si.op_word(G, 0, R, 0)], []]         # lane 2: the other tile
    racy = {(0, 0, 0, 0)}
    return [
        (prog(r1, si.SCOPE_TILE, 0b11), set()),
        (prog(r2, si.SCOPE_TILE, 0b11), racy),
        (prog(r1, si.SCOPE_TILE, 0b10), racy),          # only the other tile syncs
        (prog(r1, si.SCOPE_WAVE, 0b1), set()),
        (prog(r2, si.SCOPE_WAVE, 0b1), set()),
        (prog(r1, si.SCOPE_NONE, 0), racy),
        (prog(r2, si.SCOPE_NONE, 0), racy),
    ]


def test_nested_tiles_order_exactly_their_own_lanes():
    for prog, want in nested_closed_cases():
        assert oracle.flagged_program(prog, 64, 2) == want == brute.flagged_program(prog, 64, 2)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    subs = MUTANTS[name]
    subs = subs if isinstance(subs, list) else [subs]
    mutated = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    for pat, rep in subs:
        mutated, n = re.subn(pat, rep, mutated)
        assert n >= 1, "mutation did not apply"
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o",
                           str(so_path), str(c_path)])
    saved_so, saved_handle = oracle._SO, oracle._lib_handle
    try:
        oracle._SO, oracle._lib_handle = str(so_path), None
        assert not _pins_hold(), f"mutant {name} passes every pin"
    finally:
        oracle._SO, oracle._lib_handle = saved_so, saved_handle
    assert _pins_hold()


@pytest.mark.parametrize("tile,threads,blocks", [(2, 4, 1), (4, 4, 1), (4, 8, 2), (8, 16, 1)])
def test_tile_reduction_closed_form(tile, threads, blocks):
    """Sub-wave reduction: the oracle (waves of the tile width), the
    operational brute force (up to 4 threads) and the closed form agree for
    every dropped tile barrier."""
    from oracle import brute
    steps = (2 * tile).bit_length() - 1
    for drop in [-1] + list(range(steps)):
        prog = si.tile_reduce_program(tile, blocks, threads, drop)
        want = cf.tile_reduce_flagged(tile, blocks, threads, drop)
        assert oracle.flagged_program(prog, tile) == want, (tile, drop)
        if threads * blocks <= 4:
            assert brute.flagged_program(prog, tile) == want, (tile, drop)
    assert cf.tile_reduce_flagged(tile, blocks, threads, -1) == set()


def test_switched_off_threads_are_not_monitored():
    """Monitoring switched off in a thread (operation kind 3): its accesses
    leave the log, so races that need them are not flagged.  Oracle against
    the operational brute force on random programs with switch operations."""
    G = si.SPACE_GLOBAL
    w = si.op_word(G, 0, si.KIND_W, 0)
    r = si.op_word(G, 0, si.KIND_R, 0)
    for off in (False, True):
        first = [si.switch_word(False), w] if off else [w]
        per = [[[first, [r]]]]
        prog = si.Program([si.build_launch(1, 2, [0], [0], per)], [1], 1)
        want = set() if off else {(0, 0, 0, 0)}
        assert oracle.flagged_program(prog) == want == brute.flagged_program(prog)
    n = 0
    for s in range(60):
        prog = si.random_program(811 * s + 3, launches=2, blocks=2, threads=3, phases=3,
                                 max_ops=2, global_regions=1, global_words=2, lds_words=2,
                                 scope_p=(0.4, 0.2, 0.4), wave_width=2, p_switch=0.25)
        assert oracle.flagged_program(prog, 2) == brute.flagged_program(prog, 2), s
        n += len(oracle.flagged_program(prog, 2))
    assert n > 0
