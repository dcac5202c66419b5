"""The checker's transition function (the device code, evaluated on the host
through hr_fsm_step) against the oracle: every happens-before-consistent
processing order of a program's accesses must reach the race state at
exactly the locations the pairwise definition flags.  Also pins the paper's
worked scenarios."""
import json
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si
from fsm_replay import random_orders, replay
from paper_2401_04701_amd import hr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def widen(log, narrow):
    """Relabel threads of a log built with `narrow`-lane waves onto 64-lane
    waves: lane l of narrow wave w becomes thread 64*w + l."""
    out = log.copy()
    t = out["thread"].astype(np.int64)
    out["thread"] = ((t // narrow) * 64 + t % narrow).astype(np.uint32)
    return out


SETTINGS = [
    # blocks, threads, narrow wave width, phases, max_ops, gwords, lwords, launches
    (1, 4, 2, 3, 2, 3, 2, 2),
    (2, 2, 1, 3, 2, 3, 2, 2),
    (2, 4, 2, 4, 2, 4, 3, 3),
    (3, 3, 1, 4, 2, 2, 2, 2),
    (2, 6, 3, 3, 3, 5, 3, 2),
]


@pytest.mark.parametrize("setting", SETTINGS)
def test_fsm_flags_oracle_set_in_every_order(setting):
    blocks, threads, ww, phases, max_ops, gw, lw, launches = setting
    racy = clean = 0
    for s in range(40):
        prog = si.random_program(7919 * s + blocks * 31 + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=2, global_words=gw,
                                 lds_words=lw, kind_p=(0.5, 0.25, 0.25),
                                 scope_p=(0.25, 0.35, 0.4), wave_width=ww)
        log = oracle.model_program(prog, ww)
        want = oracle.flagged(log.copy(), ww)
        wide = widen(log, ww)
        for order in random_orders(wide, 12, seed=s):
            assert replay(wide, order) == want, (setting, s)
        touched = {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
                   for r in log}
        racy += len(want)
        clean += len(touched - want)
    assert racy > 0 and clean > 0


def test_fsm_on_litmus_programs_many_orders():
    """Larger homogeneous groups: many readers then one writer, per scope."""
    G, L = si.SPACE_GLOBAL, si.SPACE_LDS
    for space in (G, L):
        for writer_epoch in (0, 1):
            per = [[[[] for _ in range(5)] for _ in range(2)] for _ in range(2)]
            for b in range(2 if space == G else 1):
                for t in range(5):
                    per[0][b][t].append(si.op_word(space, 0, si.KIND_R, 0))
            per[writer_epoch][0][4].append(si.op_word(space, 0, si.KIND_W, 0))
            launch = si.build_launch(2, 5, [si.SCOPE_BLOCK, 0], [0, 0], per)
            prog = si.Program([launch], [4], 4)
            log = oracle.model_program(prog, 2)
            want = oracle.flagged(log.copy(), 2)
            wide = widen(log, 2)
            for order in random_orders(wide, 60, seed=writer_epoch):
                assert replay(wide, order) == want


def _thread(label):
    b, w, t = (int(ch) for ch in label[1:])
    return b, 64 * w + t


def _name(word):
    tag = word & 7
    cl = (word >> 7) & 3
    cb = (word >> 5) & 3
    if tag == hr.T_RACE:
        return "RACE"
    if tag == hr.T_MB:
        return "GREAD" if cb == 1 else "MB"
    if tag in (hr.T_MW, hr.T_MT):
        return "BREAD" if cl == 1 and (tag == hr.T_MT or cb == 1) else "MULTI"
    if tag == hr.T_ST:
        return "WRITE" if cl == 3 else ("READ" if cl == 1 else "ST")
    return "INIT"


@pytest.mark.parametrize("sc", json.load(open(os.path.join(GOLDEN, "scenarios.json")))["scenarios"],
                         ids=lambda s: s["name"])
def test_paper_scenarios(sc):
    word = 0
    kinds = {"R": hr.HR_READ, "W": hr.HR_WRITE, "A": hr.HR_ATOMIC}
    for kind, who, bc, want in sc["steps"]:
        b, t = _thread(who)
        word = hr.fsm_step(hr.HR_GLOBAL, word, kinds[kind], 0, b, t, bc, 0)
        assert _name(word) == want, (sc["name"], kind, who, want, hex(word))


def test_race_is_sticky_and_repeat_access_is_noop():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        sp = int(rng.integers(0, 2))
        args = [int(rng.integers(0, 3)), int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                int(rng.integers(0, 200)), int(rng.integers(0, 3)), int(rng.integers(0, 2))]
        kind, launch, block, thread, bc, wc = args
        if sp == hr.HR_LDS:
            launch = block = 0
        w = hr.fsm_step(sp, hr.T_RACE, kind, launch, block, thread, bc, wc)
        assert w == hr.T_RACE
        w1 = hr.fsm_step(sp, 0, kind, launch, block, thread, bc, wc)
        w2 = hr.fsm_step(sp, w1, kind, launch, block, thread, bc, wc)
        assert w1 == w2 != 0


def test_state_changes_per_epoch_are_bounded():
    """Within one launch a location changes state only a bounded number of
    times: the summary classes only grow until a new epoch starts, which
    bounds the compare-and-swap retries of contending lanes."""
    rng = np.random.default_rng(9)
    for _ in range(300):
        word, changes = 0, 0
        for _ in range(40):
            kind = int(rng.integers(0, 3))
            b, t = int(rng.integers(0, 3)), int(rng.integers(0, 130))
            new = hr.fsm_step(hr.HR_GLOBAL, word, kind, 1, b, t, 0, 0)
            changes += new != word
            word = new
        assert changes <= 8


def test_wave_group_effect_is_its_first_two_lanes():
    """Grouping lanes of one hook instruction that hit the same word: the
    lanes share kind, block, wave and both epochs and differ in thread, and
    after any reachable state every lane past the first two distinct ones
    leaves the word unchanged.  So an owner lane applying itself and one
    other member is the whole group's effect (in the order owner, other,
    rest, an order the hook may see anyway)."""
    rng = np.random.default_rng(13)
    tried = 0
    for sp in (hr.HR_GLOBAL, hr.HR_LDS):
        for _ in range(1500):
            # a reachable word: a happens-before-consistent walk of one launch
            word, bcs, wcs = 0, [0, 0, 0], {}
            for _ in range(int(rng.integers(0, 10))):
                b = int(rng.integers(0, 3)) if sp == hr.HR_GLOBAL else 0
                t = int(rng.integers(0, 192))
                if rng.random() < 0.2:
                    bcs[b] += 1
                w = (b, t >> 6, bcs[b])
                if rng.random() < 0.2:
                    wcs[w] = wcs.get(w, 0) + 1
                word = hr.fsm_step(sp, word, int(rng.integers(0, 3)), 1, b, t, bcs[b],
                                   wcs.get(w, 0))
            # one hook instruction of one wave at the current epochs
            kind = int(rng.integers(0, 3))
            b = int(rng.integers(0, 3)) if sp == hr.HR_GLOBAL else 0
            wave = int(rng.integers(0, 3))
            bc = bcs[b] + int(rng.integers(0, 2))
            wc = wcs.get((b, wave, bcs[b]), 0) if bc == bcs[b] else 0
            lanes = rng.choice(64, size=int(rng.integers(3, 7)), replace=False)
            seq = [word]
            for ln in lanes:
                seq.append(hr.fsm_step(sp, seq[-1], kind, 1, b, 64 * wave + int(ln), bc, wc))
            assert all(x == seq[2] for x in seq[3:]), (sp, hex(word), kind, lanes)
            tried += 1
    assert tried == 3000


def test_describe_decodes_each_summary_state():
    """hr_describe against summaries built by the transition function."""
    G, L = hr.HR_GLOBAL, hr.HR_LDS
    R, W, A = hr.HR_READ, hr.HR_WRITE, hr.HR_ATOMIC
    none = 0xFFFFFFFF
    st = hr.fsm_step(G, 0, R, 3, 5, 70, 2, 1)             # one thread
    d = hr.describe(G, st)
    assert d == {"state": hr.HR_S_THREAD, "class_launch": 1, "class_block": 1, "class_wave": 1,
                 "launch": 3, "block": 5, "bc": 2, "wave": 1, "wc": 1, "thread": 70}
    mt = hr.fsm_step(G, st, R, 3, 5, 71, 2, 1)            # another thread of that wave
    d = hr.describe(G, mt)
    assert d["state"] == hr.HR_S_THREADS and d["thread"] == none and d["wave"] == 1
    assert (d["class_wave"], d["block"], d["bc"], d["wc"]) == (1, 5, 2, 1)
    mw = hr.fsm_step(G, mt, A, 3, 5, 200, 2, 0)           # another wave: read + atomic race
    assert hr.describe(G, mw)["state"] == hr.HR_S_RACE
    mw = hr.fsm_step(G, mt, R, 3, 5, 200, 2, 0)
    d = hr.describe(G, mw)
    assert d["state"] == hr.HR_S_WAVES and d["wave"] == none and d["wc"] == none
    assert (d["class_block"], d["block"], d["bc"]) == (1, 5, 2)
    mb = hr.fsm_step(G, mw, R, 3, 6, 0, 0, 0)             # another block
    d = hr.describe(G, mb)
    assert d["state"] == hr.HR_S_BLOCKS and d["block"] == none and d["bc"] == none
    assert (d["launch"], d["class_block"]) == (3, 1)
    w2 = hr.fsm_step(G, st, W, 3, 5, 70, 3, 0)            # same thread, later block epoch
    d = hr.describe(G, w2)
    assert (d["state"], d["class_launch"], d["class_block"], d["bc"]) == (hr.HR_S_THREAD, 3, 3, 3)
    assert hr.describe(G, 0)["state"] == hr.HR_S_INIT
    # LDS words carry no launch, block or launch class
    ls = hr.fsm_step(L, 0, W, 0, 0, 130, 4, 2)
    d = hr.describe(L, ls)
    assert (d["state"], d["thread"], d["bc"], d["wc"], d["wave"]) == (hr.HR_S_THREAD, 130, 4, 2, 2)
    assert d["launch"] == none and d["block"] == none and d["class_launch"] == 0
    lw = hr.fsm_step(L, hr.fsm_step(L, 0, R, 0, 0, 1, 0, 0), R, 0, 0, 65, 0, 0)
    d = hr.describe(L, lw)
    assert (d["state"], d["class_block"], d["bc"]) == (hr.HR_S_WAVES, 1, 0)
    with pytest.raises(hr.HRError):
        hr.describe(L, hr.fsm_step(G, mw, R, 3, 6, 0, 0, 0) & 7)   # no multi-block LDS state


def _host_records(log, order):
    """Race records as the hook would make them, replaying `order` on the
    host: the word replaced and the completing access alone."""
    from race_records import CLASS  # noqa: F401
    words, recs = {}, []
    for i in order:
        r = log[i]
        sp, rg, ix = int(r["space"]), int(r["region"]), int(r["index"])
        b, t, L = int(r["block"]), int(r["thread"]), int(r["launch"])
        wkey = (1, rg, b, ix, L) if sp == hr.HR_LDS else (0, rg, 0, ix)
        old = words.get(wkey, 0)
        args = (int(r["kind"]), L & 511, b, t, int(r["bc"]), int(r["wc"]))
        new = hr.fsm_step(sp, old, *args)
        words[wkey] = new
        if (new & 7) == hr.T_RACE and (old & 7) != hr.T_RACE:
            rec = np.zeros(1, dtype=hr.RACE_DTYPE)[0]
            rec["space"], rec["kind"], rec["region"] = sp, int(r["kind"]), rg
            rec["block"], rec["launch"], rec["index"], rec["tid"] = b, L, ix, t
            rec["before"] = old
            rec["with"] = hr.fsm_step(sp, 0, *args)
            recs.append(rec)
    return recs


def test_race_record_check_accepts_host_records_and_rejects_planted():
    """The record validity check (used on the GPU's records) accepts the
    records a host replay makes and rejects records with a planted mistake."""
    from race_records import by_key, record_key, record_problem
    checked = rejected = 0
    for s in range(25):
        prog = si.random_program(4099 * s + 11, launches=2, blocks=2, threads=4, phases=3,
                                 max_ops=2, global_regions=2, global_words=3, lds_words=2,
                                 kind_p=(0.5, 0.25, 0.25), scope_p=(0.25, 0.35, 0.4),
                                 wave_width=2)
        log = widen(oracle.model_program(prog, 2), 2)
        keys = by_key(log)
        for order in random_orders(log, 3, seed=s):
            for rec in _host_records(log, order):
                assert record_problem(rec, keys[record_key(rec)]) is None
                checked += 1
                bad = rec.copy()
                bad["tid"] = int(rec["tid"]) ^ 1            # another thread
                rejected += record_problem(bad, keys[record_key(rec)]) is not None
                bad = rec.copy()
                bad["before"] = 0                           # an empty history cannot race
                rejected += record_problem(bad, keys[record_key(rec)]) is not None
    assert checked > 50 and rejected == 2 * checked


TILE_SETTINGS = [
    # blocks, threads, tile width, phases, max_ops, gwords, lwords, launches
    (1, 8, 2, 4, 2, 3, 2, 2),
    (2, 8, 4, 3, 2, 3, 3, 2),
    (1, 48, 16, 4, 1, 40, 24, 2),
    (2, 64, 32, 3, 1, 48, 24, 2),
    (1, 12, 4, 5, 1, 12, 8, 1),
]


@pytest.mark.parametrize("setting", TILE_SETTINGS)
def test_fsm_with_tiles_flags_oracle_set_in_every_order(setting):
    """Sub-wave synchronization: with tiles of 2^s lanes as the groups
    (wave_bits = s), barriers of a tile order only its lanes, and the machine
    must reach the oracle's set (waves of the tile width) in every
    happens-before-consistent order, with thread indices as they are."""
    blocks, threads, tw, phases, max_ops, gw, lw, launches = setting
    wb = tw.bit_length() - 1
    racy = clean = 0
    for s in range(30):
        prog = si.random_program(6151 * s + tw * 7 + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=2, global_words=gw,
                                 lds_words=lw, kind_p=(0.5, 0.25, 0.25),
                                 scope_p=(0.2, 0.55, 0.25), wave_width=tw)
        log = oracle.model_program(prog, tw)
        want = oracle.flagged(log.copy(), tw)
        for order in random_orders(log, 10, seed=s, wave_width=tw):
            assert replay(log, order, wb) == want, (setting, s)
        touched = {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
                   for r in log}
        racy += len(want)
        clean += len(touched - want)
    assert racy > 0 and clean > 0


def test_tile_barrier_orders_only_its_tile():
    """Two lanes of one wave in different 4-lane tiles: a tile barrier
    between a write and a read orders them only when both lanes are in the
    tile that synchronized."""
    G, W, R = hr.HR_GLOBAL, hr.HR_WRITE, hr.HR_READ
    w = hr.fsm_step(G, 0, W, 1, 0, 1, 0, 0, 2)                  # lane 1, tile 0, epoch 0
    same_tile = hr.fsm_step(G, w, R, 1, 0, 2, 0, 1, 2)          # lane 2 after tile 0's barrier
    other_tile = hr.fsm_step(G, w, R, 1, 0, 5, 0, 0, 2)         # lane 5 (tile 1), no barrier
    assert (same_tile & 7) != hr.T_RACE and (other_tile & 7) == hr.T_RACE
    # with whole waves the same two lanes are one group: the read of lane 5
    # after a wave barrier is ordered
    assert (hr.fsm_step(G, hr.fsm_step(G, 0, W, 1, 0, 1, 0, 0), R, 1, 0, 5, 0, 1) & 7) \
        != hr.T_RACE


# ------------------------------------------------------ tiles nested in waves
NESTED_SETTINGS = [
    # blocks, threads, tile width, phases, max_ops, gwords, lwords, launches
    (1, 8, 2, 5, 2, 3, 2, 2),
    (2, 8, 4, 4, 2, 3, 3, 2),
    (1, 96, 16, 4, 1, 40, 24, 2),     # two waves of 16-lane tiles (one partial)
    (1, 128, 8, 3, 1, 48, 24, 1),
    (1, 12, 2, 6, 1, 8, 6, 1),
]


@pytest.mark.parametrize("setting", NESTED_SETTINGS)
def test_fsm_nested_tiles_flag_oracle_set_in_every_order(setting):
    """Tiles nested in waves, each with their own barrier: the nested machine
    reaches the oracle's set (waves of 64 lanes, tiles of the given width) in
    every happens-before-consistent order, on programs mixing block, wave and
    tile barriers."""
    from fsm_replay import random_orders_nested, replay_nested
    blocks, threads, tw, phases, max_ops, gw, lw, launches = setting
    tb = tw.bit_length() - 1
    racy = clean = 0
    for s in range(30):
        prog = si.random_program(4441 * s + tw * 3 + threads, launches=launches,
                                 blocks=blocks, threads=threads, phases=phases,
                                 max_ops=max_ops, global_regions=2, global_words=gw,
                                 lds_words=lw, kind_p=(0.5, 0.25, 0.25),
                                 scope_p=(0.2, 0.2, 0.15, 0.45), tile_width=tw)
        log = oracle.model_program(prog, 64, tw)
        want = oracle.flagged(log.copy(), 64, tw)
        for order in random_orders_nested(log, 8, seed=s, tile_width=tw):
            assert replay_nested(log, order, tb) == want, (setting, s)
        touched = {(int(r["space"]), int(r["region"]), int(r["lds_block"]), int(r["index"]))
                   for r in log}
        racy += len(want)
        clean += len(touched - want)
    assert racy > 0 and clean > 0


def test_nested_merge_is_the_summary_of_the_union():
    """The fold's merge on the nested machine: merging the words two halves
    of a barrier-consistent access sequence leave (the second half applied
    to a fresh word) gives the race state exactly when the whole sequence
    races, and otherwise the word the whole sequence leaves, up to the
    identity fields that only pick which accessor is named."""
    from fsm_replay import random_orders_nested
    rng = np.random.default_rng(5)
    checked = 0
    for s in range(60):
        prog = si.random_program(77 * s + 1, launches=1, blocks=2, threads=8, phases=4,
                                 max_ops=2, global_regions=1, global_words=2, lds_words=1,
                                 p_lds=0.0, kind_p=(0.5, 0.25, 0.25),
                                 scope_p=(0.2, 0.2, 0.15, 0.45), tile_width=2)
        log = oracle.model_program(prog, 64, 2)
        for order in random_orders_nested(log, 3, seed=s, tile_width=2):
            for key in {(int(log["region"][i]), int(log["index"][i])) for i in order}:
                seq = [i for i in order if (int(log["region"][i]), int(log["index"][i])) == key]
                cut = int(rng.integers(0, len(seq) + 1))

                def run(part, start=0):
                    w = start
                    for i in part:
                        r = log[i]
                        w = hr.fsm_step_nested(0, w, int(r["kind"]), 0, int(r["block"]),
                                               int(r["thread"]), int(r["bc"]), int(r["wc"]),
                                               int(r["tc"]), 1)
                    return w
                whole = run(seq)
                # the first part as seen, then the rest as an update that
                # started from the first part's word and was overwritten
                x = run(seq[:cut])
                y = run(seq[cut:], x)
                m = hr.fsm_merge_nested(y, x, 1)
                assert ((m & 7) == hr.T_RACE) == ((whole & 7) == hr.T_RACE), (s, key, cut)
                checked += 1
    assert checked > 100


def test_describe_nested_decodes_each_summary_state():
    """hr_describe_nested against summaries the nested machine builds, tiles
    of 4 lanes (tile_bits 2) nested in 64-lane waves."""
    G, L = hr.HR_GLOBAL, hr.HR_LDS
    R, W, A = hr.HR_READ, hr.HR_WRITE, hr.HR_ATOMIC
    none = 0xFFFFFFFF

    def step(sp, old, kind, launch, block, thread, bc, wc, tc):
        return hr.fsm_step_nested(sp, old, kind, launch, block, thread, bc, wc, tc, 2)

    st = step(G, 0, R, 3, 5, 70, 2, 1, 4)                # one thread: wave 1, tile 17
    d = hr.describe_nested(G, st, 2)
    assert d == {"state": hr.HR_S_THREAD, "class_launch": 1, "class_block": 1, "class_wave": 1,
                 "class_tile": 1, "launch": 3, "block": 5, "bc": 2, "wave": 1, "wc": 1,
                 "tile": 17, "tc": 4, "thread": 70}
    mt = step(G, st, R, 3, 5, 71, 2, 1, 4)               # another thread of that tile
    d = hr.describe_nested(G, mt, 2)
    assert d["state"] == hr.HR_S_THREADS and d["thread"] == none
    assert (d["tile"], d["tc"], d["class_tile"], d["wave"], d["wc"]) == (17, 4, 1, 1, 1)
    mti = step(G, mt, R, 3, 5, 75, 2, 1, 0)              # another tile of that wave
    d = hr.describe_nested(G, mti, 2)
    assert d["state"] == hr.HR_S_TILES and d["tile"] == none and d["tc"] == none
    assert (d["wave"], d["wc"], d["class_wave"], d["block"], d["bc"]) == (1, 1, 1, 5, 2)
    assert d["class_tile"] == 0
    # a write from yet another tile of the wave in that wave epoch races
    assert hr.describe_nested(G, step(G, mti, W, 3, 5, 80, 2, 1, 0), 2)["state"] == hr.HR_S_RACE
    mw = step(G, mti, R, 3, 5, 200, 2, 0, 0)             # another wave of the block
    d = hr.describe_nested(G, mw, 2)
    assert d["state"] == hr.HR_S_WAVES and d["wave"] == none and d["wc"] == none
    assert (d["class_block"], d["class_wave"], d["block"], d["bc"]) == (1, 0, 5, 2)
    mb = step(G, mw, R, 3, 6, 0, 0, 0, 0)                # another block
    d = hr.describe_nested(G, mb, 2)
    assert d["state"] == hr.HR_S_BLOCKS and d["block"] == none and d["bc"] == none
    assert (d["launch"], d["class_block"]) == (3, 1)
    t2 = step(G, st, A, 3, 5, 70, 2, 1, 5)               # same thread, later tile epoch
    d = hr.describe_nested(G, t2, 2)
    assert (d["state"], d["class_tile"], d["class_wave"], d["tc"]) == (hr.HR_S_THREAD, 2, 3, 5)
    assert hr.describe_nested(G, 0, 2)["state"] == hr.HR_S_INIT
    # the same thread index splits into another tile number at another width
    assert hr.describe_nested(G, st, 4)["tile"] == 70 >> 4
    # LDS words carry no launch, block or launch class
    ls = step(L, 0, W, 0, 0, 130, 4, 2, 3)
    d = hr.describe_nested(L, ls, 2)
    assert (d["state"], d["thread"], d["bc"], d["wc"], d["wave"], d["tile"], d["tc"]) == \
        (hr.HR_S_THREAD, 130, 4, 2, 2, 32, 3)
    assert d["launch"] == none and d["block"] == none and d["class_launch"] == 0
    lt = step(L, step(L, 0, R, 0, 0, 1, 0, 0, 0), R, 0, 0, 5, 0, 0, 0)
    d = hr.describe_nested(L, lt, 2)
    assert (d["state"], d["wave"], d["class_wave"]) == (hr.HR_S_TILES, 0, 1)
    for bad in ((L, mb & 7, 2), (G, 7, 2), (G, st, 0), (G, st, 6), (2, st, 2)):
        with pytest.raises(hr.HRError):
            hr.describe_nested(*bad)


def _host_records_nested(log, order, tile_bits):
    """Race records of the nested machine as the hook would make them,
    replaying `order` on the host."""
    words, recs = {}, []
    for i in order:
        r = log[i]
        sp, rg, ix = int(r["space"]), int(r["region"]), int(r["index"])
        b, t, L = int(r["block"]), int(r["thread"]), int(r["launch"])
        wkey = (1, rg, b, ix, L) if sp == hr.HR_LDS else (0, rg, 0, ix)
        old = words.get(wkey, 0)
        args = (int(r["kind"]), L & 511 if sp == hr.HR_GLOBAL else 0, b, t, int(r["bc"]),
                int(r["wc"]), int(r["tc"]), tile_bits)
        new = hr.fsm_step_nested(sp, old, *args)
        words[wkey] = new
        if (new & 7) == hr.T_RACE and (old & 7) != hr.T_RACE:
            rec = np.zeros(1, dtype=hr.RACE_DTYPE)[0]
            rec["space"], rec["kind"], rec["region"] = sp, int(r["kind"]), rg
            rec["block"], rec["launch"], rec["index"], rec["tid"] = b, L, ix, t
            rec["before"] = old
            rec["with"] = hr.fsm_step_nested(sp, 0, *args)
            recs.append(rec)
    return recs


def test_nested_record_check_accepts_host_records_and_rejects_planted():
    """The record validity check in its nested form accepts every record a
    host replay of the nested machine makes, on programs mixing block, wave
    and tile barriers, and rejects each with a planted mistake (another
    thread as the completing access, an empty history, another kind)."""
    from fsm_replay import random_orders_nested
    from race_records import by_key, record_key, record_problem
    checked = rejected = 0
    for s in range(40):
        tw = (2, 4)[s % 2]
        tb = tw.bit_length() - 1
        prog = si.random_program(5231 * s + 3, launches=2, blocks=2, threads=8, phases=4,
                                 max_ops=2, global_regions=2, global_words=3, lds_words=2,
                                 kind_p=(0.5, 0.25, 0.25), scope_p=(0.2, 0.2, 0.15, 0.45),
                                 tile_width=tw)
        log = oracle.model_program(prog, 64, tw)
        keys = by_key(log)
        for order in random_orders_nested(log, 3, seed=s, tile_width=tw):
            for rec in _host_records_nested(log, order, tb):
                k = keys[record_key(rec)]
                assert record_problem(rec, k, wave_bits=tb, nested=True) is None, (s, rec)
                checked += 1
                bad = rec.copy()
                bad["tid"] = int(rec["tid"]) ^ 1
                rejected += record_problem(bad, k, wave_bits=tb, nested=True) is not None
                bad = rec.copy()
                bad["before"] = 0
                rejected += record_problem(bad, k, wave_bits=tb, nested=True) is not None
                bad = rec.copy()
                bad["kind"] = (int(rec["kind"]) + 1) % 3
                rejected += record_problem(bad, k, wave_bits=tb, nested=True) is not None
    assert checked > 50 and rejected == 3 * checked


def test_flat_table_equals_bit_logic():
    """The flat-table transition (HR_CFG_FSM_TABLE, built at compile time
    from the bit logic) equals the bit logic on every word: all eight tags
    and class fields against accesses in each relation, random raw words,
    and words reached by random access sequences; group widths 2..64."""
    rng = np.random.default_rng(17)
    n = 0
    for tag in range(8):
        for cls in range(64):
            base = tag | (cls << 3) | (int(rng.integers(0, 1 << 55)) << 9)
            for rel_args in ((1, 5, 67, 3, 2), (2, 5, 67, 3, 2), (1, 6, 67, 3, 2),
                             (1, 5, 67, 4, 2), (1, 5, 131, 3, 2), (1, 5, 67, 3, 3),
                             (1, 5, 68, 3, 2)):
                for kind in range(3):
                    for wb in (6, 3):
                        old = base if tag else 0
                        a = hr.fsm_step(hr.HR_GLOBAL, old, kind, *rel_args, wave_bits=wb)
                        assert hr.fsm_step_table(old, kind, *rel_args, wave_bits=wb) == a
                        n += 1
    for trial in range(4000):
        old = int(rng.integers(0, 2 ** 63)) * int(rng.integers(1, 3)) if trial % 2 else 0
        for _ in range(int(rng.integers(0, 4))):
            old = hr.fsm_step(hr.HR_GLOBAL, old, int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                              int(rng.integers(0, 3)), int(rng.integers(0, 200)),
                              int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                              int(rng.integers(1, 7)))
        args = (int(rng.integers(0, 3)), int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                int(rng.integers(0, 200)), int(rng.integers(0, 3)), int(rng.integers(0, 3)),
                int(rng.integers(1, 7)))
        assert hr.fsm_step_table(old, *args) == hr.fsm_step(hr.HR_GLOBAL, old, *args)
        n += 1
    assert n > 20000
    import ctypes
    out = ctypes.c_uint64(0)
    assert hr.lib().hr_fsm_step_table(hr.HR_GLOBAL, 0, 0, 0, 0, 0, 0, 0, 6,
                                      ctypes.byref(out)) == 0
    assert hr.lib().hr_fsm_step_table(hr.HR_LDS, 0, 0, 0, 0, 0, 0, 0, 6,
                                      ctypes.byref(out)) == hr.HR_E_INVAL   # global words only
