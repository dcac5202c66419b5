"""The 4-byte global shadow word (a context with HR_CFG_WORD4).  Its
transition, evaluated on the host through hr_fsm_step_word4, is checked
against the oracle and against the 8-byte word: within its field widths it
flags exactly the oracle's set in every happens-before-consistent order;
beyond them (block ids or thread indices folded) it flags a subset."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from fsm_replay import random_orders, replay
from paper_2401_04701_amd import hr
from test_fsm import SETTINGS, TILE_SETTINGS, widen

G = hr.HR_GLOBAL
# wave clock, block clock and thread widths; the block field gets 27 - 15 = 12 bits
WIDTHS = (3, 3, 9)


def program(seed, blocks, threads, ww, phases, max_ops, gw, lw, launches):
    return si.random_program(seed, launches=launches, blocks=blocks, threads=threads,
                             phases=phases, max_ops=max_ops, global_regions=2, global_words=gw,
                             lds_words=lw, kind_p=(0.5, 0.25, 0.25), scope_p=(0.25, 0.35, 0.4),
                             wave_width=ww)


@pytest.mark.parametrize("setting", SETTINGS)
def test_word4_flags_oracle_set_in_every_order(setting):
    blocks, threads, ww, phases, max_ops, gw, lw, launches = setting
    racy = 0
    for s in range(25):
        prog = program(7919 * s + blocks * 31 + threads, blocks, threads, ww, phases, max_ops,
                       gw, lw, launches)
        log = oracle.model_program(prog, ww)
        want = oracle.flagged(log.copy(), ww)
        wide = widen(log, ww)
        for order in random_orders(wide, 8, seed=s):
            assert replay(wide, order, word4=WIDTHS) == want, (setting, s)
        racy += len(want)
    assert racy > 0


@pytest.mark.parametrize("setting", TILE_SETTINGS)
def test_word4_with_tiles_flags_oracle_set_in_every_order(setting):
    """Tiles of 2^s lanes as the synchronization groups: the group bits are
    the thread field's bits from s up."""
    blocks, threads, tw, phases, max_ops, gw, lw, launches = setting
    wb = tw.bit_length() - 1
    racy = 0
    for s in range(20):
        prog = si.random_program(6151 * s + tw * 7 + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=2, global_words=gw,
                                 lds_words=lw, kind_p=(0.5, 0.25, 0.25),
                                 scope_p=(0.2, 0.55, 0.25), wave_width=tw)
        log = oracle.model_program(prog, tw)
        want = oracle.flagged(log.copy(), tw)
        for order in random_orders(log, 6, seed=s, wave_width=tw):
            assert replay(log, order, wb, word4=WIDTHS) == want, (setting, s)
        racy += len(want)
    assert racy > 0


def test_word4_widens_to_the_8byte_summary_in_all_21_states():
    """Step for step, the 4-byte word widens to the 8-byte word (launch 0)
    of the same accesses, and the walk visits every state number."""
    rng = np.random.default_rng(5)
    wcb, bcb, tb = 2, 2, 8
    seen = {0}
    for _ in range(6000):
        w4, w8 = 0, 0
        bc = wc = 0
        for _ in range(int(rng.integers(1, 10))):
            kind = int(rng.integers(0, 3))
            b = int(rng.choice([0, 0, 0, 1]))
            t = int(rng.choice([0, 1, 64]))
            if rng.random() < 0.2 and bc < 3:       # clocks move forward, as barriers do
                bc, wc = bc + 1, 0
            elif rng.random() < 0.2 and wc < 1:
                wc += 1
            w4 = hr.fsm_step_word4(w4, kind, b, t, bc, wc, 6, wcb, bcb, tb)
            w8 = hr.fsm_step(G, w8, kind, 0, b, t, bc, wc)
            assert hr.word4_widen(w4, wcb, bcb, tb) == w8
            seen.add(w4 & 31)
    assert seen == set(range(21))


def test_word4_state_numbers_decode():
    """Each of the 21 state numbers widens to a summary that hr_describe
    accepts, with the state its number range names; 21..31 are not words."""
    names = [hr.HR_S_INIT, hr.HR_S_RACE] + [hr.HR_S_BLOCKS] * 2 + [hr.HR_S_WAVES] * 4 + \
        [hr.HR_S_THREADS] * 6 + [hr.HR_S_THREAD] * 7
    for idx in range(21):
        assert hr.describe(G, hr.word4_widen(idx))["state"] == names[idx]
    for idx in range(21, 32):
        with pytest.raises(hr.HRError):
            hr.word4_widen(idx)


def test_word4_identity_fields_round_trip():
    """The fields of a single-thread summary come back through the 4-byte
    word at the edges of their widths (block folded to its field)."""
    wcb, bcb, tb = 1, 2, 8                          # block field 16 bits
    for b, t, bc, wc in [(0, 0, 0, 0), (65535, 255, 3, 1), (65536 + 7, 3, 1, 0),
                         (12345, 128, 2, 1)]:
        w4 = hr.fsm_step_word4(0, hr.HR_WRITE, b, t, bc, wc, 6, wcb, bcb, tb)
        d = hr.describe(G, hr.word4_widen(w4, wcb, bcb, tb))
        assert (d["state"], d["block"], d["thread"], d["bc"], d["wc"]) == \
            (hr.HR_S_THREAD, b % 65536, t, bc, wc)
        assert d["launch"] == 0


def test_word4_rejects_clocks_beyond_their_fields():
    with pytest.raises(hr.HRError):
        hr.fsm_step_word4(0, 0, 0, 0, 4, 0, 6, 1, 2, 8)     # bc 4 in a 2-bit field
    with pytest.raises(hr.HRError):
        hr.fsm_step_word4(0, 0, 0, 0, 0, 2, 6, 1, 2, 8)     # wc 2 in a 1-bit field
    with pytest.raises(hr.HRError):
        hr.fsm_step_word4(0, 0, 0, 0, 0, 0, 6, 1, 2, 11)    # thread field above 10 bits


@pytest.mark.parametrize("case", ["threads", "blocks"])
def test_word4_beyond_its_widths_flags_a_subset(case):
    """Folded thread indices (a 6-bit thread field: lanes of different
    waves look alike) or folded block ids (a 3-bit block field, ten blocks)
    can hide races and never add one."""
    if case == "threads":
        widths, shape = (3, 3, 6), (2, 4, 2, 3, 2, 3, 2, 1)
    else:
        widths, shape = (6, 8, 10), (10, 2, 1, 3, 2, 3, 2, 1)
    blocks, threads, ww, phases, max_ops, gw, lw, launches = shape
    strict = racy = 0
    for s in range(30):
        prog = program(104729 * s + 17, blocks, threads, ww, phases, max_ops, gw, lw, launches)
        log = oracle.model_program(prog, ww)
        want = oracle.flagged(log.copy(), ww)
        wide = widen(log, ww)
        for order in random_orders(wide, 4, seed=s):
            got = replay(wide, order, word4=widths)
            assert got <= want, (case, s)
            strict += got != want
        racy += len(want)
    assert racy > 0
    if case == "threads":
        assert strict > 0


def test_word4_folded_blocks_hide_their_race():
    """Blocks 0 and 8 share a folded id in a 3-bit block field: their
    threads 0 writing one word look like one thread, so the race is missed,
    while the default 16-bit block field tells them apart."""
    narrow, wide = (6, 8, 10), (1, 2, 8)
    w = hr.fsm_step_word4(0, hr.HR_WRITE, 0, 0, 0, 0, 6, *narrow)
    assert hr.fsm_step_word4(w, hr.HR_WRITE, 8, 0, 0, 0, 6, *narrow) != hr.T_RACE
    w = hr.fsm_step_word4(0, hr.HR_WRITE, 0, 0, 0, 0, 6, *wide)
    assert hr.fsm_step_word4(w, hr.HR_WRITE, 8, 0, 0, 0, 6, *wide) == hr.T_RACE
