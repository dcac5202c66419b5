"""CPU model of the device hook protocol under adversarial interleavings.

Test helper.  Every instrumented access of a barrier program runs the same
sequence of shared-memory steps as the HIP hook, each step atomic on its own:

  global: load -> (transition) -> exchange -> [fold: merge + compare-and-swap]*
  LDS:    load -> [transition + compare-and-swap]*

A random scheduler interleaves the steps of all threads (one step at a time),
subject to barrier semantics: a thread passes a block barrier only when every
thread of its block has reached it with its hooks finished; likewise for wave
barriers.  The transition and merge are the library's own functions
(hr_fsm_step, hr_fsm_merge), evaluated on the host.  The result is the set
of keys for which a race record was appended, and the final shadow words.
"""
from __future__ import annotations

import numpy as np

import synth_inputs as si
from paper_2401_04701_amd import hr

RACE = hr.T_RACE


class _Thread:
    __slots__ = ("block", "thread", "wave", "tile", "ops", "pc", "bc", "wc", "tc", "hook")

    def __init__(self, block, thread, wave, ops, tile=0):
        self.block, self.thread, self.wave, self.ops, self.tile = block, thread, wave, ops, tile
        self.pc, self.bc, self.wc, self.tc, self.hook = 0, 0, 0, 0, None


def _expand(launch, narrow, tiles=False, nested=0):
    """Per-thread op lists: ('A', space, region, index, kind) / ('B',) / ('W',)
    / ('T',).  Threads of `narrow`-lane waves are relabelled onto 64-lane
    waves, or, with `tiles`, keep their index and the groups are tiles of
    `narrow` lanes.  With `nested` (a tile width), threads keep their index
    in 64-lane waves and tiles of `nested` lanes have barriers of their own
    (scope 3)."""
    threads = []
    for b in range(launch.blocks):
        for t in range(launch.threads):
            w = t // (64 if nested else narrow)
            g = t // nested if nested else 0
            ops = []
            for p in range(launch.phases):
                for word in launch.thread_ops(p, b, t):
                    space, region, kind, index = si.op_fields(word)
                    ops.append(("A", space, region, index, kind))
                sc = int(launch.scope[p])
                if sc == si.SCOPE_BLOCK:
                    ops.append(("B",))
                elif sc == si.SCOPE_WAVE and (int(launch.wave_mask[p]) >> w) & 1:
                    ops.append(("W",))
                elif (sc == si.SCOPE_TILE and nested and g < 64 and
                      (int(launch.wave_mask[p]) >> g) & 1):
                    ops.append(("T",))
            label = t if (tiles or nested) else w * 64 + t % narrow
            threads.append(_Thread(b, label, w, ops, g))
    return threads


STATS = {"folds": 0, "fold_rounds": 0}


def simulate(program, narrow: int, seed: int, tiles: bool = False, nested: int = 0,
             blind: float = 0.0):
    """tiles: the checker synchronizes tiles of `narrow` lanes (wave_bits =
    log2 narrow) instead of relabelling them onto 64-lane waves.  nested: a
    tile width; the nested machine (hr_fsm_step_nested / hr_fsm_merge_nested)
    with tiles of that many lanes inside 64-lane waves, each level with its
    own barriers and clock.  blind: the probability that a global hook
    skips its load and steps from the initial word instead (the blind
    exchange: publish the access alone, then fold back what it replaced)."""
    rng = np.random.default_rng(seed)
    wb = int(narrow).bit_length() - 1 if tiles else 6
    if nested:
        wb = int(nested).bit_length() - 1
    gwords = {}
    pushed = []
    for L, launch in enumerate(program.launches):
        lwords = {}
        ths = _expand(launch, narrow, tiles, nested)
        by_block, by_wave, by_tile = {}, {}, {}
        for th in ths:
            by_block.setdefault(th.block, []).append(th)
            by_wave.setdefault((th.block, th.wave), []).append(th)
            by_tile.setdefault((th.block, th.tile), []).append(th)
        while True:
            # release barriers whose groups have fully arrived, repeatedly
            released = True
            while released:
                released = False
                for grp, kind in ((by_block, "B"), (by_wave, "W"), (by_tile, "T")):
                    for members in grp.values():
                        if all(m.hook is None and m.pc < len(m.ops) and m.ops[m.pc][0] == kind
                               for m in members):
                            released = True
                            for m in members:
                                m.pc += 1
                                if kind == "B":
                                    m.bc += 1
                                    m.wc = m.tc = 0
                                elif kind == "W":
                                    m.wc += 1
                                    m.tc = 0
                                else:
                                    m.tc += 1
            runnable = [th for th in ths if th.hook is not None or
                        (th.pc < len(th.ops) and th.ops[th.pc][0] == "A")]
            if not runnable:
                assert all(th.pc == len(th.ops) for th in ths), "barrier deadlock"
                break
            th = runnable[int(rng.integers(0, len(runnable)))]
            _micro_step(th, L, gwords, lwords, pushed, wb, bool(nested),
                        blind > 0 and rng.random() < blind)
    return pushed, gwords


def _step(space, old, kind, L, th, wb, nested):
    if nested:
        return hr.fsm_step_nested(space, old, kind, L & 511 if space == hr.HR_GLOBAL else 0,
                                  th.block if space == hr.HR_GLOBAL else 0, th.thread, th.bc,
                                  th.wc, th.tc, wb)
    if space == hr.HR_GLOBAL:
        return hr.fsm_step(space, old, kind, L & 511, th.block, th.thread, th.bc, th.wc, wb)
    return hr.fsm_step(space, old, kind, 0, 0, th.thread, th.bc, th.wc, wb)


def _merge(x, y, wb, nested):
    return hr.fsm_merge_nested(x, y, wb) if nested else hr.fsm_merge(x, y, wb)


def _micro_step(th, L, gwords, lwords, pushed, wb=6, nested=False, blind=False):
    if th.hook is None:
        _, space, region, index, kind = th.ops[th.pc]
        th.hook = {"space": space, "region": region, "index": index, "kind": kind,
                   "stage": "load", "blind": blind}
    h = th.hook
    if h["space"] == si.SPACE_GLOBAL:
        key = (0, h["region"], 0, h["index"])
        if h["stage"] == "load":
            old = 0 if h["blind"] else gwords.get(key, 0)
            nw = _step(hr.HR_GLOBAL, old, h["kind"], L, th, wb, nested)
            if nw == old:
                return _done(th)
            h.update(stage="xchg", old=old, nw=nw)
            return
        if h["stage"] == "xchg":
            r = gwords.get(key, 0)
            gwords[key] = h["nw"]
            if h["nw"] == RACE:
                if r != RACE:
                    pushed.append(key)
                return _done(th)
            if r == h["old"]:
                return _done(th)
            h.update(stage="fold", cur=h["nw"], lost=r)
            STATS["folds"] += 1
            return
        if h["stage"] == "fold":
            STATS["fold_rounds"] += 1
            m = _merge(h["cur"], h["lost"], wb, nested)
            if m == h["cur"]:
                return _done(th)
            seen = gwords.get(key, 0)
            if seen == h["cur"]:
                gwords[key] = m
                if m == RACE and h["lost"] != RACE:
                    pushed.append(key)
                return _done(th)
            h["cur"] = seen
            return
    else:
        wkey = (th.block, h["region"], h["index"])
        key = (1, h["region"], th.block, h["index"])
        if h["stage"] == "load":
            h.update(stage="cas", old=lwords.get(wkey, 0))
            return
        nw = _step(hr.HR_LDS, h["old"], h["kind"], L, th, wb, nested)
        if nw == h["old"]:
            return _done(th)
        seen = lwords.get(wkey, 0)
        if seen == h["old"]:
            lwords[wkey] = nw
            if nw == RACE:
                pushed.append(key)
            return _done(th)
        h["old"] = seen


def _done(th):
    th.hook = None
    th.pc += 1
