"""Schedule brute force -- test infrastructure, not part of the checker.

An operational statement of the race definition (paper, Sec. II-A), written
independently of the pairwise check in ``oracle.c``: every interleaving of a
tiny straight-line barrier program is explored, and a location races when
some reachable state has two different threads whose next operations are
conflicting accesses to it (both could execute next, in either order).

Barrier semantics (Sec. II-B): a thread that reaches a block barrier waits
until every thread of its block is at that barrier; a wave barrier waits for
every thread of the wave; a tile barrier (groups below the wave, which the
paper leaves to future work, Sec. VI) waits for every thread of the tile.
Launches run one after another, so only accesses of one launch can be
pending together.  Lanes of one wave are interleaved freely: lockstep
execution gives no ordering.

State spaces grow as (ops+1)^threads, so this is for programs with a handful
of threads (the two-thread argument of Sec. II-B says races in barrier-only
programs already show up with two threads).
"""
from __future__ import annotations

from collections import deque

import synth_inputs as si


def _conflict(k1: int, k2: int) -> bool:
    # not both plain reads, not both atomics
    return not (k1 == k2 and k1 != si.KIND_W)


def thread_lists(launch, wave_width: int, tile_width: int = 0):
    """Per-thread operation lists: ('A', key, kind), ('B',), ('W',) or
    ('T',) (a tile barrier: tiles of tile_width lanes nested in the waves)."""
    progs = {}
    for b in range(launch.blocks):
        for t in range(launch.threads):
            lst = []
            w = t // wave_width
            g = t // tile_width if tile_width else 0
            on = True                      # kind 3 switches monitoring off / on
            for p in range(launch.phases):
                for word in launch.thread_ops(p, b, t):
                    space, region, kind, index = si.op_fields(word)
                    if kind == si.KIND_SWITCH:
                        on = bool(index & 1)
                        continue
                    if not on:
                        continue
                    key = (space, region, b if space == si.SPACE_LDS else 0, index)
                    lst.append(("A", key, kind))
                sc = int(launch.scope[p])
                if sc == si.SCOPE_BLOCK:
                    lst.append(("B",))
                elif sc == si.SCOPE_WAVE and w < 64 and (int(launch.wave_mask[p]) >> w) & 1:
                    lst.append(("W",))
                elif (sc == si.SCOPE_TILE and tile_width and g < 64 and
                      (int(launch.wave_mask[p]) >> g) & 1):
                    lst.append(("T",))
            progs[(b, t)] = lst
    return progs


def flagged_launch(launch, wave_width: int = 64, max_states: int = 2_000_000,
                   tile_width: int = 0) -> set:
    progs = thread_lists(launch, wave_width, tile_width)
    tids = sorted(progs)
    lists = [progs[t] for t in tids]
    n = len(tids)
    block_of = [t[0] for t in tids]
    wave_of = [(t[0], t[1] // wave_width) for t in tids]
    tile_of = [(t[0], t[1] // tile_width) if tile_width else None for t in tids]
    members_block = {}
    members_wave = {}
    members_tile = {}
    for i in range(n):
        members_block.setdefault(block_of[i], []).append(i)
        members_wave.setdefault(wave_of[i], []).append(i)
        if tile_width:
            members_tile.setdefault(tile_of[i], []).append(i)

    def nxt(state, i):
        pc = state[i]
        return lists[i][pc] if pc < len(lists[i]) else None

    racy = set()
    start = tuple([0] * n)
    seen = {start}
    todo = deque([start])
    while todo:
        st = todo.popleft()
        pending = [(i, nxt(st, i)) for i in range(n)]
        acc = [(i, op) for i, op in pending if op is not None and op[0] == "A"]
        # race check in this state
        for x in range(len(acc)):
            for y in range(x + 1, len(acc)):
                (i, oi), (j, oj) = acc[x], acc[y]
                if oi[1] == oj[1] and _conflict(oi[2], oj[2]):
                    racy.add(oi[1])
        succ = []
        for i, op in acc:
            s2 = list(st)
            s2[i] += 1
            succ.append(tuple(s2))
        # barriers: release a group when all its members wait at one
        for grp, kind in ((members_block, "B"), (members_wave, "W"), (members_tile, "T")):
            for members in grp.values():
                if all(pending[i][1] is not None and pending[i][1][0] == kind
                       for i in members):
                    s2 = list(st)
                    for i in members:
                        s2[i] += 1
                    succ.append(tuple(s2))
        for s2 in succ:
            if s2 not in seen:
                seen.add(s2)
                if len(seen) > max_states:
                    raise RuntimeError("state space too large for brute force")
                todo.append(s2)
    return racy


def flagged_program(program, wave_width: int = 64, tile_width: int = 0) -> set:
    out = set()
    for launch in program.launches:
        out |= flagged_launch(launch, wave_width, tile_width=tile_width)
    return out
