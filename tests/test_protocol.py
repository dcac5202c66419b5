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
