"""The hook protocol (coherent load, exchange, fold-back merge for global
memory; compare-and-swap for LDS) under adversarial interleavings of its
atomic steps must report exactly the oracle's flagged set, whatever the
schedule.  Runs the library's transition and merge functions on the host."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
import protocol_sim as ps

SETTINGS = [
    # blocks, threads, narrow wave, phases, max_ops, gwords, lwords, launches, kind_p
    (1, 4, 2, 2, 3, 2, 2, 2, (0.5, 0.25, 0.25)),
    (2, 3, 1, 3, 2, 2, 2, 2, (0.5, 0.25, 0.25)),
    (3, 3, 3, 2, 3, 3, 2, 2, (0.7, 0.1, 0.2)),
    (2, 4, 2, 3, 2, 2, 2, 3, (0.45, 0.1, 0.45)),
    (4, 2, 1, 2, 3, 1, 1, 2, (0.6, 0.05, 0.35)),
    (1, 6, 3, 3, 2, 2, 2, 2, (0.8, 0.05, 0.15)),
]


def _keys(log):
    return {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
            for r in log}


@pytest.mark.parametrize("setting", SETTINGS)
def test_protocol_reports_oracle_set_under_any_schedule(setting):
    blocks, threads, ww, phases, max_ops, gw, lw, launches, kp = setting
    folds0 = ps.STATS["folds"]
    racy = clean = 0
    for s in range(30):
        prog = si.random_program(104729 * s + 17 * blocks + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=1, global_words=gw,
                                 lds_words=lw, kind_p=kp, scope_p=(0.4, 0.3, 0.3),
                                 wave_width=ww)
        log = oracle.model_program(prog, ww)
        want = oracle.flagged(log.copy(), ww)
        for sched in range(25):
            pushed, words = ps.simulate(prog, ww, seed=1000 * s + sched)
            assert set(pushed) == want, (setting, s, sched)
            race_words = {k for k, w in words.items() if w == ps.RACE}
            assert race_words == {k for k in want if k[0] == 0}
        racy += len(want)
        clean += len(_keys(log) - want)
    assert racy > 0 and clean > 0
    assert ps.STATS["folds"] > folds0, "schedules never exercised the fold-back path"


@pytest.mark.parametrize("blind", [0.5, 1.0])
@pytest.mark.parametrize("setting", SETTINGS[:4])
def test_protocol_blind_exchanges_report_oracle_set(setting, blind):
    """Global hooks that skip their load and publish the access alone (the
    word a fresh location would get), then fold back the word the exchange
    replaced: under any schedule the flagged set is still the oracle's.  The
    merge keeps a newer block or wave epoch's detail over an older one of
    the same block or wave, which makes a summary of everything before as
    good a starting point as the current word."""
    blocks, threads, ww, phases, max_ops, gw, lw, launches, kp = setting
    folds0 = ps.STATS["folds"]
    racy = 0
    for s in range(20):
        prog = si.random_program(7919 * s + 31 * blocks + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=1, global_words=gw,
                                 lds_words=lw, kind_p=kp, scope_p=(0.4, 0.3, 0.3),
                                 p_lds=0.2, wave_width=ww)
        log = oracle.model_program(prog, ww)
        want = oracle.flagged(log.copy(), ww)
        for sched in range(20):
            pushed, words = ps.simulate(prog, ww, seed=500 * s + sched, blind=blind)
            assert set(pushed) == want, (setting, blind, s, sched)
            race_words = {k for k, w in words.items() if w == ps.RACE}
            assert race_words == {k for k in want if k[0] == 0}
        racy += len(want)
    assert racy > 0 and ps.STATS["folds"] > folds0


def test_protocol_contended_single_location():
    """Many threads of several blocks, waves and epochs on one or two words:
    the exchange overwrites concurrent updates constantly."""
    folds0 = ps.STATS["folds"]
    for s in range(40):
        prog = si.random_program(s, launches=2, blocks=3, threads=4, phases=3, max_ops=2,
                                 global_regions=1, global_words=2, lds_words=1,
                                 p_lds=0.1, kind_p=(0.6, 0.1, 0.3) if s % 2 else (0.0, 0.0, 1.0),
                                 scope_p=(0.3, 0.3, 0.4), wave_width=2)
        want = oracle.flagged_program(prog, 2)
        for sched in range(20):
            pushed, _ = ps.simulate(prog, 2, seed=s * 100 + sched)
            assert set(pushed) == want, (s, sched)
    assert ps.STATS["folds"] - folds0 > 50


@pytest.mark.parametrize("tw", [2, 4])
def test_protocol_with_tiles_reports_oracle_set(tw):
    """The exchange + fold protocol with tiles of `tw` lanes as the groups."""
    folds0 = ps.STATS["folds"]
    for s in range(30):
        prog = si.random_program(7919 * s + tw, launches=2, blocks=2, threads=2 * tw,
                                 phases=3, max_ops=2, global_regions=1, global_words=2,
                                 lds_words=2, kind_p=(0.5, 0.2, 0.3), scope_p=(0.3, 0.45, 0.25),
                                 wave_width=tw)
        log = oracle.model_program(prog, tw)
        want = oracle.flagged(log.copy(), tw)
        for sched in range(20):
            pushed, _ = ps.simulate(prog, tw, seed=100 * s + sched, tiles=True)
            assert set(pushed) == want, (tw, s, sched)
    assert ps.STATS["folds"] > folds0


@pytest.mark.parametrize("tile,threads", [(2, 8), (4, 8), (2, 66)])
def test_protocol_nested_tiles_reports_oracle_set(tile, threads):
    """The exchange + fold protocol on the nested machine: tiles of `tile`
    lanes with their own barriers inside 64-lane waves (66 threads: a
    second, partial wave), interleaved with wave and block barriers; every
    schedule reports the oracle's nested set."""
    folds0 = ps.STATS["folds"]
    for s in range(12 if threads > 8 else 30):
        prog = si.random_program(104729 * s + tile + threads, launches=2, blocks=2,
                                 threads=threads, phases=4, max_ops=1 if threads > 8 else 2,
                                 global_regions=1, global_words=2, lds_words=2,
                                 kind_p=(0.5, 0.2, 0.3), scope_p=(0.2, 0.2, 0.15, 0.45),
                                 tile_width=tile)
        want = oracle.flagged_program(prog, 64, tile)
        for sched in range(12):
            pushed, _ = ps.simulate(prog, 64, seed=100 * s + sched, nested=tile)
            assert set(pushed) == want, (tile, threads, s, sched)
    assert ps.STATS["folds"] > folds0


# --------------------------------------------------------------------------
# The hooks as the tuned kernels issue them (protocol_pipe.py): preloaded
# words, split issue and settle, and wave grouping, each and together.
import protocol_pipe as pp

PIPE_MODES = [
    # name, preload depth, split (pending settles), grouping width
    ("preload", 2, 0, 0),
    ("split", 0, 2, 0),
    ("group64", 0, 0, 64),
    ("group2", 0, 0, 2),
    ("all", 2, 2, 0),
    ("preload_group", 1, 0, 4),
]


def _pipe_programs(base, n, dense=False):
    """Sparse-race programs (many words, few operations, most of them reads
    or atomics), so that one lost update changes the verdict of some key;
    dense: one 8-lane wave per block, so that grouped hooks form."""
    out = []
    for s in range(n):
        args = dict(launches=2, blocks=2, threads=4, phases=3, max_ops=2, global_regions=1,
                    global_words=6, lds_words=2, kind_p=(0.6, 0.15, 0.25), p_lds=0.2,
                    scope_p=(0.4, 0.3, 0.3), wave_width=2)
        if dense:
            args.update(threads=8, wave_width=8, global_words=3, kind_p=(0.7, 0.1, 0.2),
                        p_lds=0.1)
        out.append(si.random_program(base + 7 * s, **args))
    return out


def _directed_programs():
    """One wave of four lanes: only grouped accesses carry the races."""
    R, W, A = si.KIND_R, si.KIND_W, si.KIND_A

    def g(kind, idx=0):
        return si.op_word(si.SPACE_GLOBAL, 0, kind, idx)

    def prog(phase0, phase1=None, scopes=(0, 0)):
        phases = [[phase0]] + ([[phase1]] if phase1 is not None else [])
        launch = si.build_launch(1, 4, list(scopes[:len(phases)]), [1] * len(phases), phases)
        return si.Program([launch], [2], 2)
    return [
        # four lanes read, then lane 0 writes in the same wave epoch: a race
        # that only a read by another lane of the group exposes
        prog([[g(R), g(W)], [g(R)], [g(R)], [g(R)]]),
        # the same with a wave barrier before the write: no race
        prog([[g(R)], [g(R)], [g(R)], [g(R)]], [[g(W)], [], [], []], scopes=(1, 0)),
        # four lanes write at once
        prog([[g(W)], [g(W)], [g(W)], [g(W)]]),
        # four lanes' atomics, then lane 2 reads in the same epoch
        prog([[g(A)], [g(A)], [g(A), g(R)], [g(A)]]),
        # two words, reads grouped on one, a write on the other
        prog([[g(R, 1)], [g(R, 1)], [g(R, 1), g(W, 0)], [g(R, 1), g(R, 0)]]),
    ]


def _check_pipe(progs, ww, depth, split, width, scheds, seed0=0):
    for i, prog in enumerate(progs):
        want = oracle.flagged(oracle.model_program(prog, ww).copy(), ww)
        for sched in range(scheds):
            pushed, words = pp.simulate(prog, ww, seed=seed0 + 97 * i + sched, preload=depth,
                                        split=split, group_width=width)
            # (a key may be recorded more than once: an exchange computed from
            # an older word can briefly replace a race state before its fold
            # restores it, and another hook may record the key again in that
            # window; the report removes duplicates, and the set is exact)
            assert set(pushed) == want, (i, sched)
            assert {k for k, w in words.items() if w == pp.RACE} == \
                {k for k in want if k[0] == 0}


@pytest.mark.parametrize("mode", PIPE_MODES, ids=lambda m: m[0])
def test_pipelined_hooks_report_oracle_set(mode):
    """Every schedule of the pipelined hooks reports the oracle's set and
    leaves exactly the racy global words in the race state; the fold path
    runs in every mode, and each mode's own behaviour (a preloaded word
    missing the thread's own update, several hooks in flight, a grouped
    update) shows up."""
    name, depth, split, width = mode
    s0 = dict(pp.STATS)
    progs = _pipe_programs(1000 + len(name), 30, dense=bool(width))
    ww = 8 if width else 2
    racy = sum(len(oracle.flagged(oracle.model_program(p, ww).copy(), ww)) for p in progs)
    keys = sum(len({(int(r["space"]), int(r["index"])) for r in oracle.model_program(p, ww)})
               for p in progs)
    assert 0 < racy < keys                      # racy and clean locations both occur
    _check_pipe(progs, ww, depth, split, width, 10)
    if width:
        _check_pipe(_directed_programs(), 4, depth, split, width, 40)
    d = {k: pp.STATS[k] - s0[k] for k in pp.STATS}
    assert d["folds"] > 0, d
    if depth:
        assert d["stale_own"] > 0, d
    if split:
        assert d["split_overlaps"] > 0, d
    if width:
        assert d["grouped"] > 0 and d["partners"] > 0, d


def test_pipelined_checks_catch_planted_mistakes(monkeypatch):
    """The same programs and checks fail on a model with a mistake planted:
    a grouped update that forgets its partner's access, or an exchange that
    overwrote an update and never folds it back."""
    def caught(progs, ww, **kw):
        try:
            _check_pipe(progs, ww, scheds=10, **kw)
        except AssertionError:
            return True
        return False

    orig_expand = pp._expand

    def partner_lost(launch, narrow, width, rng):
        ths = orig_expand(launch, narrow, width, rng)
        for th in ths:
            for op in th.ops:
                if op[0] == "A" and len(op[5]) == 2:
                    del op[5][1:]
        return ths
    monkeypatch.setattr(pp, "_expand", partner_lost)
    assert caught(_directed_programs(), 4, depth=0, split=0, width=64)
    monkeypatch.setattr(pp, "_expand", orig_expand)

    def no_fold(th, f, gwords, pushed):
        th.done.add(th.pending.pop(0)["pos"])
    monkeypatch.setattr(pp, "_fold_step", no_fold)
    progs = _pipe_programs(1000, 30)
    for depth, split in ((2, 0), (0, 2), (0, 0)):
        assert caught(progs, 2, depth=depth, split=split, width=0), (depth, split)
def test_pipelined_duplicate_edges_fold_their_own_stale_words():
    """One thread hits one word with atomics, then reads and writes it,
    back to back (consecutive duplicate edges, a seeded edge among them),
    while another thread of another block does the same: with every word
    preloaded two accesses ahead and two exchanges in flight the verdict is
    still the oracle's."""
    s0 = pp.STATS["stale_own"]
    for s in range(20):
        prog = si.random_program(5000 + s, launches=2, blocks=2, threads=1, phases=2,
                                 max_ops=5, global_regions=1, global_words=1, lds_words=1,
                                 p_lds=0.0, kind_p=(0.3, 0.2, 0.5), scope_p=(1.0, 0.0, 0.0),
                                 wave_width=1)
        want = oracle.flagged_program(prog, 1)
        for sched in range(15):
            pushed, _ = pp.simulate(prog, 1, seed=s * 31 + sched, preload=2, split=2)
            assert set(pushed) == want, (s, sched)
    assert pp.STATS["stale_own"] > s0
